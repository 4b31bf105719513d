// gfx950 kernels for the two-step Lax-Wendroff evolution of the homogeneous
// (2+1)D Teukolsky equation (arXiv:1010.3816, Sec. 3, Eqs. (lw1)-(lw2)).
//
// Fused step kernel.  One wavefront owns a tile of 64 consecutive r*
// columns (62 output columns plus one halo column on each side) and a chunk
// of theta rows, which it sweeps row by row:
//   * stage 1 (Eq. lw1) is evaluated once per half point and row: lane L
//     averages its column with the column of lane L+1 (the averaging of the
//     printed kernel_average1) and forms u^{n+1/2}_{i+1/2};
//   * stage 2 (Eq. lw2) at column i combines the stage-1 values of lanes
//     L-1 and L; both neighbour exchanges are cross-lane moves, so the
//     stage-1 field never leaves registers;
//   * the theta stencil of S (2nd-order centred differences) needs rows
//     j-1, j, j+1 of the averaged fields; a three-row register window slides
//     along theta, and the pole ghost rows (mirror for even |m|, anti-mirror
//     for odd |m|) are formed in registers by a wavefront-uniform branch;
//   * Phi = Pi = 0 is written on the radial boundary columns.
// Every input point is read once per tile (plus a 2-column and 2-row halo),
// every output point written once; the coefficients of Eq. (1) are rebuilt
// per point from 1-D radial tables (per lane, held in registers) and 1-D
// angular tables (per row, wavefront-uniform), so no 2-D coefficient array
// is streamed from HBM.
//
// Extraction is fused: the wavefront whose tile contains the bilinear
// stencil of an extraction point accumulates Phi of the INPUT state while
// it streams the rows, and writes the sample at the end of its sweep.
#include "internal.hpp"

namespace teuk {
namespace {

struct cd {
    double re, im;
};

__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd cavg(cd a, cd b) { return {0.5 * (a.re + b.re), 0.5 * (a.im + b.im)}; }

// Cross-lane moves: lane L receives the value held by lane L+1 / lane L-1,
// as two 32-bit DPP wavefront shifts (wave_shl:1 / wave_shr:1).  The edge
// lanes (63 and 0) receive 0; their results are never stored.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kRowsInFlight = 3;  // rows of input loaded ahead of the row being finished
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) { return dpp_move<kDppWaveShl1>(v); }
__device__ __forceinline__ double from_left(double v) { return dpp_move<kDppWaveShr1>(v); }
__device__ __forceinline__ cd from_right(cd v) { return {from_right(v.re), from_right(v.im)}; }
__device__ __forceinline__ cd from_left(cd v) { return {from_left(v.re), from_left(v.im)}; }

// The coefficients of the first-order system at one (position, row), with
// the difference-operator scalings folded in: a2s = A2/dth^2, a1s = A1/(2 dth).
struct Coef {
    double b, cre, cim, ctr, cti, a2s, a1s, v0r, v0i;
};

struct Rad {
    double rho, rho2, a2d, rb1, rb2, rb3, ctr, cti0, cti1, b1n, dl2, v0r, v0i;
};

struct Ang {
    double sn2, cs, cotp, pd;
};

__device__ __forceinline__ Rad load_rad(const double* rad, int pitch, int kind, int pos) {
    auto f = [&](int field) { return rad[((size_t)field * 2 + kind) * pitch + pos]; };
    Rad R;
    R.rho = f(R_RHO);
    R.rho2 = f(R_RHO2);
    R.a2d = f(R_A2D);
    R.rb1 = f(R_RB1);
    R.rb2 = f(R_RB2);
    R.rb3 = f(R_RB3);
    R.ctr = f(R_CTR);
    R.cti0 = f(R_CTI0);
    R.cti1 = f(R_CTI1);
    R.b1n = f(R_B1N);
    R.dl2 = f(R_DL2);
    R.v0r = f(R_V0R);
    R.v0i = f(R_V0I);
    return R;
}

__device__ __forceinline__ Ang load_ang(const double* ang, int nth, int j) {
    Ang G;
    G.sn2 = ang[A_SN2 * nth + j];
    G.cs = ang[A_CS * nth + j];
    G.cotp = ang[A_COTP * nth + j];
    G.pd = ang[A_PD * nth + j];
    return G;
}

// 1/Sigma and 1/Sigma^2 at one (position, row).
struct Sig {
    double isig, inv;
};

__device__ __forceinline__ Sig kerr_sigma(const Rad& R, const Ang& G) {
    const double sig2 = fma(-R.a2d, G.sn2, R.rho2);
    const double inv = 1.0 / sig2;
    return {sqrt(inv), inv};
}

// Eq. (1) coefficients from the factored tables (see RadField / AngField).
__device__ __forceinline__ Coef kerr_coef(const Rad& R, const Ang& G, Sig s) {
    Coef c;
    c.b = R.rho * s.isig;
    const double bp = s.isig * fma(-fma(-R.rb3, G.sn2, R.rb2), s.inv, R.rb1);
    c.ctr = R.ctr * s.inv;
    c.cti = fma(R.cti1, G.cs, R.cti0) * s.inv;
    const double b1 = R.b1n * s.inv;
    c.cre = fma(c.b, bp - c.ctr, -b1);
    c.cim = -c.b * c.cti;
    c.a2s = R.dl2 * s.inv;
    c.a1s = c.a2s * G.cotp;
    c.v0r = fma(R.dl2, G.pd, R.v0r) * s.inv;
    c.v0i = R.v0i * s.inv;
    return c;
}

__device__ __forceinline__ Coef user_coef(const double* u, int nth, int pitch, int j, int pos, double inv_dth2,
                                          double inv_2dth) {
    auto f = [&](int k) { return u[((size_t)k * nth + j) * pitch + pos]; };
    Coef c;
    c.b = f(U_B);
    c.cre = f(U_CRE);
    c.cim = f(U_CIM);
    c.ctr = f(U_CTRE);
    c.cti = f(U_CTIM);
    c.a2s = f(U_A2) * inv_dth2;
    c.a1s = f(U_A1) * inv_2dth;
    c.v0r = f(U_V0RE);
    c.v0i = f(U_V0IM);
    return c;
}

// Pi row of S:  -Ct q + A2 (f_{j+1} - 2 f_j + f_{j-1})/dth^2
//               + A1 (f_{j+1} - f_{j-1})/(2 dth) - V0 f_j
__device__ __forceinline__ cd s_pi(const Coef& k, cd fm, cd f0, cd fp, cd q) {
    const double lr = (fp.re + fm.re) - 2.0 * f0.re;
    const double li = (fp.im + fm.im) - 2.0 * f0.im;
    const double gr = fp.re - fm.re;
    const double gi = fp.im - fm.im;
    double sr = fma(k.a2s, lr, k.a1s * gr);
    double si = fma(k.a2s, li, k.a1s * gi);
    sr -= fma(k.ctr, q.re, -k.cti * q.im);
    si -= fma(k.ctr, q.im, k.cti * q.re);
    sr -= fma(k.v0r, f0.re, -k.v0i * f0.im);
    si -= fma(k.v0r, f0.im, k.v0i * f0.re);
    return {sr, si};
}

// D applied to (dP, dQ), Pi row:  c dP - b dQ.
__device__ __forceinline__ cd d_pi(const Coef& k, cd dP, cd dQ) {
    return {fma(k.cre, dP.re, fma(-k.cim, dP.im, -k.b * dQ.re)),
            fma(k.cre, dP.im, fma(k.cim, dP.re, -k.b * dQ.im))};
}

// Workgroups are dispatched round-robin over the 8 XCDs; map them so that
// each XCD (own L2) receives a contiguous range of tiles, i.e. neighbouring
// strips whose halo columns overlap.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int x = b % X, idx = b / X, per = nb / X, rem = nb % X;
    return x * per + min(x, rem) + idx;
}

// Loads always read a valid (clamped) address; where the column lies
// outside the grid the value is zeroed by a bit mask at its point of use, so
// the load itself is unconditional and stays in flight until it is needed.
__device__ __forceinline__ cd ld(const double2* __restrict__ p, size_t o) {
    const double2 v = p[o];
    return {v.x, v.y};
}

__device__ __forceinline__ cd masked(cd v, unsigned long long mask) {
    return {__longlong_as_double(__double_as_longlong(v.re) & mask),
            __longlong_as_double(__double_as_longlong(v.im) & mask)};
}

typedef double v2d __attribute__((ext_vector_type(2)));

// Streaming store of one complex value (16 B, one dwordx4 per lane): the
// new state is not read again by this launch.
__device__ __forceinline__ void st(double2* p, size_t o, cd v) {
    v2d w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<v2d*>(p + o));
}

// All pointers are distinct allocations (restrict): the uniform reads of
// the angular tables and extraction descriptors become scalar loads.
template <bool KERR>
__global__ void __launch_bounds__(512)
    lw_step_kernel(const double2* __restrict__ phi_in, const double2* __restrict__ pi_in,
                   double2* __restrict__ phi_out, double2* __restrict__ pi_out, const double* __restrict__ rad,
                   const double* __restrict__ ang, const double* __restrict__ uci, const double* __restrict__ uch,
                   const ExtPoint* __restrict__ ext, double2* __restrict__ series, StepScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    // wavefront-uniform tile index, made explicit so that everything derived
    // from it (rows, table reads, loop control) is scalar
    const int tile = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * wpb + (threadIdx.x / kWave));
    if (tile >= A.n_tiles) return;
    const int strip = tile % A.n_strips;
    const int chunk = tile / A.n_strips;
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols - 1 + lane;
    const unsigned long long in = ((col >= 0) && (col < nr)) ? ~0ull : 0ull;
    const int ci = min(max(col, 0), nr - 1);  // clamped integer column
    const int hi = min(max(col, 0), nr - 2);  // clamped half point col + 1/2
    const bool store_ok = (lane >= 1) && (lane <= kWave - 2) && (col < nr);
    const bool boundary = (col == 0) || (col == nr - 1);
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const double sg = (double)A.sigma;
    const int last = (j1 < nth) ? j1 : nth - 1;  // last row this tile reads

    Rad Ri, Rh;
    if constexpr (KERR) {
        Ri = load_rad(rad, P, 0, ci);
        Rh = load_rad(rad, P, 1, hi);
    }

    // extraction point owned by this lane, if any
    int my_e = -1, my_ra = -1, my_rb = -1;
    double my_wr = 0.0, my_wa = 0.0, my_wb = 0.0;
    cd acc = {0.0, 0.0};
    for (int e = 0; e < A.n_ext; ++e) {
        const ExtPoint E = ext[e];
        const int es = E.col / kStripCols;
        if (es == strip && E.rowa / A.rows == chunk && lane == E.col - es * kStripCols + 1) {
            my_e = e;
            my_ra = E.rowa;
            my_rb = E.rowb;
            my_wr = E.wr;
            my_wa = E.wa;
            my_wb = E.wb;
        }
    }

    // ---- per-row stage-1 pieces -------------------------------------------
    // fresh(t): from u(t) of this lane and of lane L+1:
    //   ubar (Phi, Pi), delta (Phi, Pi) at the half point to the right,
    //   h_Phi there, and (via lane L-1) hbar_Phi, dh_Phi at this column.
    struct Row {
        cd p, q;          // u(t) at this column
        cd ubp, ubq, dp, dq;
        cd hbp, dhp;      // average / difference of h_Phi of the two neighbouring halves
        Sig sh;           // 1/Sigma at (half, t)
    };

    auto fresh = [&](int t, cd p, cd q) -> Row {
        p = masked(p, in);
        q = masked(q, in);
        Row R;
        R.p = p;
        R.q = q;
        const cd pr = from_right(p), qr = from_right(q);
        R.ubp = cavg(p, pr);
        R.ubq = cavg(q, qr);
        R.dp = csub(pr, p);
        R.dq = csub(qr, q);
        double bh;
        if constexpr (KERR) {
            const Ang G = load_ang(ang, nth, t);
            R.sh = kerr_sigma(Rh, G);
            bh = Rh.rho * R.sh.isig;
        } else {
            R.sh = {0.0, 0.0};
            bh = uch[((size_t)U_B * nth + t) * P + hi];
        }
        // h_Phi = ubar_Phi - dt/2 (b delta_Phi / dr - ubar_Pi)
        const double tb = A.hdt_dr * bh;
        const cd hp = {fma(-tb, R.dp.re, fma(A.hdt, R.ubq.re, R.ubp.re)),
                       fma(-tb, R.dp.im, fma(A.hdt, R.ubq.im, R.ubp.im))};
        const cd hpl = from_left(hp);
        R.hbp = cavg(hp, hpl);
        R.dhp = csub(hp, hpl);
        if (my_e >= 0) {
            const double w = (t == my_ra ? my_wa : 0.0) + (t == my_rb ? my_wb : 0.0);
            const cd v = {fma(my_wr, pr.re - p.re, p.re), fma(my_wr, pr.im - p.im, p.im)};
            acc.re = fma(w, v.re, acc.re);
            acc.im = fma(w, v.im, acc.im);
        }
        return R;
    };

    // ---- prologue ----------------------------------------------------------
    cd ubp_m, hbp_m;  // averaged Phi fields at row t-1
    Row cur;
    {
        if (j0 > 0) {
            const size_t o = (size_t)(j0 - 1) * P + ci;
            const Row rm = fresh(j0 - 1, ld(phi_in, o), ld(pi_in, o));
            ubp_m = rm.ubp;
            hbp_m = rm.hbp;
        }
        const size_t o = (size_t)j0 * P + ci;
        cur = fresh(j0, ld(phi_in, o), ld(pi_in, o));
        if (j0 == 0) {
            ubp_m = cscale(sg, cur.ubp);
            hbp_m = cscale(sg, cur.hbp);
        }
    }
    // Ring of D row buffers: buffer u holds row t+1 when row t (t - j0 = u
    // mod D) is finished, and is refilled with row t+1+D right after.  The
    // loop is unrolled by D so that loaded registers are never copied (a copy
    // would have to wait for the load), keeping D rows in flight.
    cd bp[kRowsInFlight], bq[kRowsInFlight];
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
        const size_t o = (size_t)min(j0 + 1 + u, last) * P + ci;
        bp[u] = ld(phi_in, o);
        bq[u] = ld(pi_in, o);
    }

    auto finish_row = [&](int t, cd& rp, cd& rq) {
        // row t+1: streamed, or the pole ghost row
        Row nxt;
        cd ubp_p, hbp_p;
        if (t + 1 < nth) {
            nxt = fresh(t + 1, rp, rq);
            ubp_p = nxt.ubp;
            hbp_p = nxt.hbp;
        } else {
            ubp_p = cscale(sg, cur.ubp);
            hbp_p = cscale(sg, cur.hbp);
        }
        {
            const size_t o = (size_t)min(t + 1 + kRowsInFlight, last) * P + ci;
            rp = ld(phi_in, o);
            rq = ld(pi_in, o);
        }

        // stage 1, Pi component at (half, t)
        Coef kh, ki;
        if constexpr (KERR) {
            const Ang G = load_ang(ang, nth, t);
            kh = kerr_coef(Rh, G, cur.sh);
            ki = kerr_coef(Ri, G, kerr_sigma(Ri, G));
        } else {
            kh = user_coef(uch, nth, P, t, hi, A.inv_dth2, A.inv_2dth);
            ki = user_coef(uci, nth, P, t, ci, A.inv_dth2, A.inv_2dth);
        }
        // h_Pi = ubar_Pi - dt/2 [ (c delta_Phi - b delta_Pi)/dr - S_Pi(ubar) ]
        const cd dq1 = d_pi(kh, cur.dp, cur.dq);
        const cd s1 = s_pi(kh, ubp_m, cur.ubp, ubp_p, cur.ubq);
        const cd hq = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, cur.ubq.re)),
                       fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, cur.ubq.im))};
        const cd hql = from_left(hq);
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);

        // stage 2 at (i, t)
        //   Phi' = Phi - dt [ b dh_Phi / dr - hbar_Pi ]
        //   Pi'  = Pi  - dt [ (c dh_Phi - b dh_Pi)/dr - S_Pi(hbar) ]
        const double tb = A.dt_dr * ki.b;
        cd np = {fma(-tb, cur.dhp.re, fma(A.dt, hbq.re, cur.p.re)),
                 fma(-tb, cur.dhp.im, fma(A.dt, hbq.im, cur.p.im))};
        const cd dq2 = d_pi(ki, cur.dhp, dhq);
        const cd s2 = s_pi(ki, hbp_m, cur.hbp, hbp_p, hbq);
        cd nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, cur.q.re)),
                 fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, cur.q.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
        }
        if (store_ok) {
            const size_t o = (size_t)t * P + col;
            st(phi_out, o, np);
            st(pi_out, o, nq);
        }

        ubp_m = cur.ubp;
        hbp_m = cur.hbp;
        if (t + 1 < nth) cur = nxt;
    };

    // whole groups of kRowsInFlight rows, then the ragged tail
    int t0 = j0;
    for (; t0 + kRowsInFlight <= j1; t0 += kRowsInFlight) {
#pragma unroll
        for (int u = 0; u < kRowsInFlight; ++u) finish_row(t0 + u, bp[u], bq[u]);
    }
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u)
        if (t0 + u < j1) finish_row(t0 + u, bp[u], bq[u]);

    if (my_e >= 0 && series != nullptr) {
        double2 w;
        w.x = acc.re;
        w.y = acc.im;
        series[my_e] = w;
    }
}

__global__ void import_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int nr, int nth,
                              int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= pitch || j >= nth) return;
    double2 v;
    v.x = 0.0;
    v.y = 0.0;
    if (i > 0 && i < nr - 1) v = src[(size_t)j * nr + i];
    dst[(size_t)j * pitch + i] = v;
}

__global__ void export_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int nr, int nth,
                              int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nr || j >= nth) return;
    dst[(size_t)j * nr + i] = src[(size_t)j * pitch + i];
}

__global__ void extract_kernel(const double2* __restrict__ phi, int pitch, const ExtPoint* __restrict__ pts,
                               int n, double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const ExtPoint E = pts[e];
    auto row = [&](int j) {
        const double2 a = phi[(size_t)j * pitch + E.col];
        const double2 b = phi[(size_t)j * pitch + E.col + 1];
        return cd{fma(E.wr, b.x - a.x, a.x), fma(E.wr, b.y - a.y, a.y)};
    };
    const cd va = row(E.rowa);
    cd v = {E.wa * va.re, E.wa * va.im};
    if (E.rowb >= 0) {
        const cd vb = row(E.rowb);
        v.re = fma(E.wb, vb.re, v.re);
        v.im = fma(E.wb, vb.im, v.im);
    }
    double2 w;
    w.x = v.re;
    w.y = v.im;
    out[e] = w;
}

__global__ void nonfinite_kernel(const double2* __restrict__ phi, const double2* __restrict__ pi, int nr, int nth,
                                 int pitch, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nr || j >= nth) return;
    const size_t o = (size_t)j * pitch + i;
    const double2 a = phi[o], b = pi[o];
    if (!isfinite(a.x) || !isfinite(a.y) || !isfinite(b.x) || !isfinite(b.y)) *flag = 1;
}

__global__ void pitch_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int rows, int cols,
                                  int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= pitch || j >= rows) return;
    dst[(size_t)j * pitch + i] = (i < cols) ? src[(size_t)j * cols + i] : 0.0;
}

}  // namespace

hipError_t launch_step(const StepArgs& a, bool kerr, int waves_per_block, hipStream_t s) {
    const int nb = (a.k.n_tiles + waves_per_block - 1) / waves_per_block;
    const dim3 block(kWave * waves_per_block), grid(nb);
    auto kern = kerr ? lw_step_kernel<true> : lw_step_kernel<false>;
    hipLaunchKernelGGL(kern, grid, block, 0, s, a.phi_in, a.pi_in, a.phi_out, a.pi_out, a.rad, a.ang, a.uci, a.uch,
                       a.ext, a.series, a.k);
    return hipGetLastError();
}

hipError_t launch_import(const double2* src, double2* dst, int nr, int nth, int pitch, hipStream_t s) {
    const dim3 block(256), grid((pitch + 255) / 256, nth);
    hipLaunchKernelGGL(import_kernel, grid, block, 0, s, src, dst, nr, nth, pitch);
    return hipGetLastError();
}

hipError_t launch_export(const double2* src, double2* dst, int nr, int nth, int pitch, hipStream_t s) {
    const dim3 block(256), grid((nr + 255) / 256, nth);
    hipLaunchKernelGGL(export_kernel, grid, block, 0, s, src, dst, nr, nth, pitch);
    return hipGetLastError();
}

hipError_t launch_extract(const double2* phi, int pitch, int /*sigma*/, const ExtPoint* pts, int n, double2* out,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 block(64), grid((n + 63) / 64);
    hipLaunchKernelGGL(extract_kernel, grid, block, 0, s, phi, pitch, pts, n, out);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const double2* phi, const double2* pi, int nr, int nth, int pitch, int* flag,
                            hipStream_t s) {
    const dim3 block(256), grid((nr + 255) / 256, nth);
    hipLaunchKernelGGL(nonfinite_kernel, grid, block, 0, s, phi, pi, nr, nth, pitch, flag);
    return hipGetLastError();
}

hipError_t launch_pitch_copy(const double* src, double* dst, int rows, int cols, int pitch, hipStream_t s) {
    const dim3 block(256), grid((pitch + 255) / 256, rows);
    hipLaunchKernelGGL(pitch_copy_kernel, grid, block, 0, s, src, dst, rows, cols, pitch);
    return hipGetLastError();
}

}  // namespace teuk
