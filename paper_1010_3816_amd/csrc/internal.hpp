// Internal declarations shared by the host library (teuk_api.cpp) and the
// gfx950 kernels (lw_kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace teuk {

// Output columns per wavefront strip.  A wavefront's 64 lanes hold the 64
// consecutive columns c0-1 .. c0+62 of its strip; lane L computes the
// stage-1 value at the half point to the right of its column, so the
// columns c0 .. c0+61 (lanes 1..62) have both neighbouring half points.
constexpr int kWave = 64;
constexpr int kStripCols = kWave - 2;
// Output columns per strip of the two-step kernel: its second step needs the
// first step's results one column further out on each side, so lanes 2..61
// hold the output columns c0 .. c0+59 of a strip whose lanes hold c0-2 .. c0+61.
constexpr int kStripCols2 = kWave - 4;

// Radial table fields, each a row of `pitch` doubles, first for the integer
// positions r*_i then for the half positions r*_{i+1/2}.  With r, Delta,
// rho = r^2 + a^2 at the position (Sigma^2 = rho^2 - a^2 Delta sin^2 th):
enum RadField : int {
    R_RHO = 0,  // rho
    R_RHO2,     // rho^2
    R_A2D,      // a^2 Delta                     Sigma^2 = rho^2 - a^2 Delta sin^2
    R_RB1,      // 2 r Delta / rho               b' = (RB1 - (RB2 - RB3 sin^2)/Sigma^2)/Sigma
    R_RB2,      // 2 r rho Delta
    R_RB3,      // a^2 (r - 1) Delta
    R_CTR,      // 2 s (r Delta - (r^2 - a^2))   Re Ct = CTR / Sigma^2
    R_CTI0,     // 4 a m r                       Im Ct = (CTI0 + CTI1 cos) / Sigma^2
    R_CTI1,     // 2 s a Delta
    R_B1N,      // rho (6 Delta/r + 2 s (r-1) + 2 r Delta/rho)     B1 = B1N / Sigma^2
    R_DL2,      // Delta / dth^2                 A2/dth^2 = DL2 / Sigma^2
    R_V0R,      // -m^2 a^2 - 6 Delta ((s+2) r^2 - (s+3) r + a^2) / r^2
    R_V0I,      // -2 s m a (r - 1)              Im V0 = V0I / Sigma^2
    kNumRad
};

// Angular table fields, stored row by row: [ntheta][kNumAng] doubles, so
// that one scalar load fetches all fields of a row.
enum AngField : int {
    A_SN2 = 0,  // sin^2 th
    A_CS,       // cos th
    A_COTP,     // cot th * dth / 2               A1/(2 dth) = A2/dth^2 * COTP
    A_PD,       // ((m + s cos th)^2 / sin^2 th - s) * dth^2   Re V0 = (DL2 PD + V0R)/Sigma^2
    kNumAng
};

// USER-mode coefficient order (matches TEUK_NCOEF in teuk.h).
enum UserCoef : int { U_B = 0, U_CRE, U_CIM, U_CTRE, U_CTIM, U_A2, U_A1, U_V0RE, U_V0IM, kNumUser };

// One extraction point: bilinear weights between columns col, col+1 and the
// rows rowa, rowb (rowb < 0: single row, ghost rows folded into the weights).
struct ExtPoint {
    int32_t col, rowa, rowb, pad;
    double wr, wa, wb, pad2;
};

// Scalar launch parameters of the step kernel (passed by value).
struct StepScalars {
    int32_t nr, nth, pitch, sigma;
    int32_t rows, n_strips, n_chunks, n_ext;
    int32_t zero;               // always 0 (an opaque row offset of LDS reads)
    int32_t keep;               // 1: the new state is written with ordinary stores (selects the kernel instance)
    int32_t order;              // two-step pass: tile order (kTileOrder*)
    int32_t bsteps;             // block pass: steps per launch
    int32_t bcols;              // block pass: columns a workgroup holds (bsteps halo columns each side)
    int32_t pad_;
    int64_t row0;               // block pass: series row of the launch's first input state (-1: not sampled)
    int64_t plane;              // nth * pitch: offset of the Pi plane in a state
    double dt, hdt, dt_dr, hdt_dr;
    double inv_dth2, inv_2dth;  // USER mode scalings
    // source term (inhomogeneous variant): time factors of the pass's steps,
    // sf[4s .. 4s+3] = f(t_n), f(t_n + dt/2) (re, im) of its step s = 0, 1
    double sf[8];
};

// Tile order of the single-grid two-step pass.  Dispatch: tile = workgroup
// x waves + wave, strips fastest; workgroups go round-robin over the 8 XCDs.
// XCD strips: each XCD takes one contiguous run of strips (its 1/8) in every
// theta chunk, so neighbouring strips (which share halo columns and 128-byte
// lines) and the chunks of a strip (which share the radial tables) meet in
// one L2; strips fastest (kTileOrderXcdStrip) or chunks fastest
// (kTileOrderXcdChunk) within the XCD.
constexpr int kTileOrderDispatch = 0, kTileOrderXcdStrip = 1, kTileOrderXcdChunk = 2;

struct StepArgs {
    const double2* u_in;     // state: [Phi, Pi][nth][pitch]
    double2* u_out;
    const double* rad;       // [kNumRad][2][pitch] (KERR)
    const double* ang;       // [nth][kNumAng]      (KERR)
    const double* uci;       // [kNumUser][nth][pitch] (USER, integer positions)
    const double* uch;       // [kNumUser][nth][pitch] (USER, half positions)
    const ExtPoint* ext;     // [n_ext]
    double2* series;         // n_ext samples of the input Phi, or nullptr
    double2* win;            // copy of the input state (two-step kernel: the intermediate state), or nullptr
    double2* series_mid;     // two-step kernel: samples of Phi after the first step, or nullptr
    const double2* src_i;    // source profile at the integer positions, [nth][pitch], or nullptr
    const double2* src_h;    // source profile at the half positions, [nth][pitch]
    StepScalars k;
};

// One member of a batched launch (device-resident descriptor).
struct BatchMember {
    double2* u[2];           // the member's two state buffers
    const double* rad;       // its radial and angular tables (KERR)
    const double* ang;
    StepScalars k;           // its launch scalars (rows shared by all members)
    int32_t tile_begin;      // first tile of this member in the work list
    int32_t tile_begin2;     // the same in the two-step work list
    int32_t n_strips2;       // its strips of the two-step kernel
    int32_t pad;
};

// One extraction point of a batched evolution: the member's two state
// buffers (the current one is selected by the batch parity) and its point.
struct BatchExtPoint {
    const double2* u[2];
    int32_t pitch, pad;
    ExtPoint e;
};

// Mode sum at observers: up to kMaxModes modes and kMaxObservers points.
constexpr int kMaxModes = 64;
constexpr int kMaxObservers = 64;
struct AssembleArgs {
    int32_t n_modes, n_obs;
    int32_t m[kMaxModes];
    double phi[kMaxObservers], r3[kMaxObservers];
};

// Scalar launch parameters of the adjoint kernel.
struct AdjScalars {
    int32_t nr, nth, pitch, sigma;
    int32_t rows, n_strips, n_chunks, zero;  // zero: always 0 (an opaque row offset of LDS reads)
    int64_t plane;                           // nth * pitch: offset of the Pi plane in a state
    int32_t n_ext;                           // extraction points (fused transposed extraction)
    int32_t keep;                            // 1: lam_out and the tangent step's state with ordinary stores
                                             // (selects the kernel instance)
    double dt, hdt, dt_dr, hdt_dr;
};

struct AdjArgs {
    const double2* nu_in;    // lambda^{m+1}, [Phi, Pi][nth][pitch]
    const double2* u_in;     // u^m
    double2* lam_out;        // lambda^m
    const double* rad;       // [kNumRad][2][pitch]
    const double* rad_da;    // d/da of rad
    const double* ang;       // [nth][kNumAng]
    double* slots;           // [n_strips * n_chunks] spin-gradient partial sums (accumulated)
    const ExtPoint* ext;     // [n_ext] extraction points
    const double* gsample;   // gradient of the output state's sample, 2 doubles per point, or nullptr
    AdjScalars k;
};

// Launchers (lw_kernels.hip, adjoint_kernels.hip).  All return the
// hipError_t of the launch.
hipError_t launch_step(const StepArgs& a, bool kerr, int waves_per_block, hipStream_t s);
// Two steps in one pass (k.n_strips counted in kStripCols2-column strips).
hipError_t launch_step2(const StepArgs& a, bool kerr, int waves_per_block, hipStream_t s);
// Small grids (ntheta <= kMaxBlockRows, Kerr coefficients): k.bsteps steps in
// one launch, each workgroup holding k.bcols columns x all rows in LDS
// (a.series: samples of the launch's input states, rows k.row0 + s).
constexpr int kMaxBlockRows = 64;
constexpr int kMaxBlockExt = 8;
constexpr int kMaxBlockSteps = 31;  // (64 columns - 2) / 2
hipError_t launch_block(const StepArgs& a, hipStream_t s);
// Zero n ints (a fill kernel: usable where a memset node is not).
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// two = true: two steps per launch (work list of tile_begin2 / n_strips2).
// keep: the members' next states with ordinary stores (StepScalars::keep).
hipError_t launch_batch(const BatchMember* members, int n_members, int total_tiles, int parity, int n_blocks,
                        int waves_per_block, bool two, bool keep, hipStream_t s);
hipError_t launch_import(const double2* src, double2* u, int f, int nr, int nth, int pitch, hipStream_t s);
hipError_t launch_export(const double2* u, double2* dst, int f, int nr, int nth, int pitch, hipStream_t s);
hipError_t launch_extract(const double2* u, int pitch, const ExtPoint* pts, int n, double2* out, hipStream_t s);
hipError_t launch_batch_extract(const BatchExtPoint* pts, int n, int parity, double2* out, hipStream_t s);
hipError_t launch_assemble(const AssembleArgs& a, int64_t n_samples, const double2* samples, double2* psi,
                           hipStream_t s);
hipError_t launch_nonfinite(const double2* u, int nr, int nth, int pitch, int* flag, hipStream_t s);
// Records `step` in *first (if still 0) when the state holds a non-finite value.
hipError_t launch_nonfinite_step(const double2* u, int nr, int nth, int pitch, long long* first, int64_t step,
                                 hipStream_t s);
// Adjoint kernel variants: cotangents only (u_in, rad_da and slots are not
// read); with the spin gradient recomputed from u^m = u_in; with the spin
// gradient as the dot product of nu with T_m = u_in, the stored tangent.
enum class AdjMode { kCotangent, kSpin, kTangentDot };
hipError_t launch_adjoint(const AdjArgs& a, int waves_per_block, AdjMode mode, hipStream_t s);
// Two cotangent adjoint steps: nu_in = lambda^{m+2} -> lam_out = lambda^m
// (k.n_strips counted in kStripCols2-column strips); a.gsample is the sample
// gradient added to lambda^{m+1}, gsample_b the one added to lambda^m.  With
// a.u_in = T_{m+1} and tan_b = T_m (stored tangents) the kernel also adds the
// spin gradient's dot products of both steps to a.slots.
hipError_t launch_adjoint2(const AdjArgs& a, const double* gsample_b, const double2* tan_b, int waves_per_block,
                           hipStream_t s);
// One step u_in -> u_out that also writes T = (dA/da) u_in to t_out (tiles of
// a.k: kStripCols-column strips, a.k.rows rows; a.rad_da the a-derivative tables).
hipError_t launch_tangent(const double2* u_in, double2* u_out, double2* t_out, const AdjArgs& a, int waves_per_block,
                          hipStream_t s);
// One step of the state and of its a-derivative v (u_in, v_in -> u_out,
// v_out; tiles as launch_tangent), with the samples of u_in and v_in at the
// first a.k.n_ext extraction points (at most one per tile; series_u/v may be
// nullptr).
hipError_t launch_spin_tangent(const double2* u_in, const double2* v_in, double2* u_out, double2* v_out,
                               double2* series_u, double2* series_v, const AdjArgs& a, int waves_per_block,
                               hipStream_t s);
// *out += sum Re(conj(g_i) t_i) over count complex values (stream order).
hipError_t launch_series_dot(const double2* g, const double2* t, int64_t count, double* out, hipStream_t s);
hipError_t launch_extract_adjoint(double2* lam, int pitch, const ExtPoint* pts, int n, const double2* g,
                                  hipStream_t s);
hipError_t launch_reduce_slots(const double* slots, int n, double* out, hipStream_t s);
hipError_t launch_zero_radial_boundary(double2* u, int nr, int nth, int pitch, hipStream_t s);
hipError_t launch_pitch_copy(const double* src, double* dst, int rows, int cols, int pitch, hipStream_t s);

}  // namespace teuk
