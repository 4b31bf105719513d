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
#include "device_common.hpp"

namespace teuk {
namespace {
// The source term of the inhomogeneous variant at one point: f g, with the
// time factor f = (fr, fi) of the stage and the profile g at the position.
__device__ __forceinline__ cd source(gin_t g, size_t o, double fr, double fi) {
    const cd v = ld(g, o);
    return {fma(fr, v.re, -fi * v.im), fma(fr, v.im, fi * v.re)};
}

// Row-sweep of one tile.  Per row t the sweep keeps:
//   p, q      Phi, Pi at (i, t)
//   ubp       stage-1 average of Phi at the half point i+1/2
//   hbp, dhp  mean and difference of the stage-1 Phi values at i-1/2, i+1/2
//   x, wp     the stage-1 Pi value at (i+1/2, t) except for its row-(t+1)
//             term: h_Pi(t) = x + wp * ubp(t+1); the theta stencil is the only
//             part of Eq. (lw1) that needs the next row.
struct Row {
    cd p, q, ubp, hbp, dhp, x;
    double wp;
    Ang g;  // angular factors of row t (wavefront-uniform, KERR)
};

// One tile (strip of 64 columns x theta chunk) of one grid.  Inlined into
// the single-grid kernel and into the batched kernel.
// KEEP: the cache policy of the new state's stores (0 streaming, 1 keeping).
template <bool KERR, bool SRC, int KEEP>
__device__ __forceinline__ void sweep_tile(gin_t __restrict__ u_in, gout_t __restrict__ u_out, ctab_t rad, ctab_t ang,
                                           ctab_t uci, ctab_t uch, cext_t ext, double2* __restrict__ series,
                                           gout_t __restrict__ win, const StepScalars& A, int strip, int chunk,
                                           int lane, gin_t __restrict__ src_i = nullptr,
                                           gin_t __restrict__ src_h = nullptr) {
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols - 1 + lane;
    // Lanes outside the grid read the clamped edge column.  Their values
    // reach only the radial boundary columns of the output, which are set to
    // zero, so they need no masking.
    const int ci = min(max(col, 0), nr - 1);  // clamped integer column
    const int hi = min(max(col, 0), nr - 2);  // clamped half point col + 1/2

    // radial factors of this lane's column and half point, held in registers
    Rad Ri, Rh;
    if constexpr (KERR) {
        Ri = load_rad(rad, P, 0, ci);
        Rh = load_rad(rad, P, 1, hi);
    }

    const bool store_ok = (lane >= 1) && (lane <= kWave - 2) && (col < nr);
    const bool boundary = (col == 0) || (col == nr - 1);
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const double sg = (double)A.sigma;
    const int last = (j1 < nth) ? j1 : nth - 1;  // last row this tile reads

    // The prologue's rows (j0-1, or row 0 again for the first tile, and j0)
    // and the ring's first rows, loaded right after the radial factors so
    // that the latencies overlap at the start of the tile.
    cd hp[2], hq[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const size_t o = (size_t)max(j0 - 1 + k, 0) * P + ci;
        hp[k] = ld(u_in, o);
        hq[k] = ld(u_in, o + A.plane);
    }
    // Ring of D row buffers: buffer u holds row t+1 when row t (t - j0 = u
    // mod D) is finished, and is refilled with row t+1+D right after.  The
    // loop is unrolled by D so that loaded registers are never copied (a copy
    // would have to wait for the load), keeping D rows in flight.
    cd bp[kRowsInFlight], bq[kRowsInFlight];
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
        const size_t o = (size_t)min(j0 + 1 + u, last) * P + ci;
        bp[u] = ld(u_in, o);
        bq[u] = ld(u_in, o + A.plane);
    }

    // the (at most one) extraction point of this tile, in scalar registers
    int e_id = -1, e_lane = 0, e_ra = -1, e_rb = -1;
    double e_wr = 0.0, e_wa = 0.0, e_wb = 0.0;
    for (int e = 0; e < A.n_ext; ++e) {
        const ExtPoint E = {ext[e].col, ext[e].rowa, ext[e].rowb, 0, ext[e].wr, ext[e].wa, ext[e].wb, 0.0};
        const int es = E.col / kStripCols;
        if (es == strip && E.rowa / A.rows == chunk) {
            e_id = e;
            e_lane = E.col - es * kStripCols + 1;
            e_ra = E.rowa;
            e_rb = E.rowb;
            e_wr = E.wr;
            e_wa = E.wa;
            e_wb = E.wb;
        }
    }
    cd acc = {0.0, 0.0};

    // angular factors of row t (clamped to the grid: rows past the last
    // are loaded ahead but never used)
    auto ang_row = [&](int t) -> Ang {
        Ang G{};
        if constexpr (KERR) G = load_ang(ang, nth, min(t, nth - 1));
        return G;
    };
    auto half_coef = [&](int t, const Ang& G, double& b) -> Coef {
        Coef k;
        if constexpr (KERR) {
            k = kerr_coef(Rh, G, kerr_sigma(Rh, G));
        } else {
            k = user_coef(uch, nth, P, t, hi, A.inv_dth2, A.inv_2dth);
        }
        b = k.b;
        return k;
    };
    auto half_b = [&](int t, const Ang& G) -> double {
        if constexpr (KERR) {
            return Rh.rho * kerr_sigma(Rh, G).isig;
        } else {
            return uch[((size_t)U_B * nth + t) * P + hi];
        }
    };

    // Stage-1 pieces of row t from u(t) of this lane and of lane L+1.
    // FULL: also the Pi part x, wp (needs ubp(t-1): `ubp_prev`, or the ghost
    // row when t == 0).  Halo rows only need ubp and hbp.
    auto fresh = [&](int t, cd p, cd q, cd ubp_prev, bool full, const Ang& G) -> Row {
        Row R;
        R.p = p;
        R.q = q;
        R.g = G;
        const cd pr = from_right(p), qr = from_right(q);
        R.ubp = cavg(p, pr);
        const cd ubq = cavg(q, qr);
        const cd dp = csub(pr, p);
        double bh;
        Coef kh;
        if (full)
            kh = half_coef(t, G, bh);
        else
            bh = half_b(t, G);
        // h_Phi = ubar_Phi - dt/2 (b delta_Phi / dr - ubar_Pi)
        const double tb = A.hdt_dr * bh;
        const cd hp = {fma(-tb, dp.re, fma(A.hdt, ubq.re, R.ubp.re)), fma(-tb, dp.im, fma(A.hdt, ubq.im, R.ubp.im))};
        const cd hpl = from_left(hp);
        R.hbp = cavg(hp, hpl);
        R.dhp = csub(hp, hpl);
        if (full) {
            // h_Pi = ubar_Pi - dt/2 [ (c delta_Phi - b delta_Pi)/dr - S_Pi(ubar) ], with
            // S_Pi(ubar) = -Ct ubar_Pi + A2 lap + A1 grad - V0 ubar_Phi split as
            // (everything but the row-(t+1) term) + (A2/dth^2 + A1/(2 dth)) ubar_Phi(t+1)
            const cd dq = csub(qr, q);
            const cd um = (t == 0) ? cscale(sg, R.ubp) : ubp_prev;
            const cd dq1 = d_pi(kh, dp, dq);
            cd s1 = s_pi(kh, um, R.ubp, cd{0.0, 0.0}, ubq);
            if constexpr (SRC) s1 = cadd(s1, source(src_h, (size_t)t * P + hi, A.sf[0], A.sf[1]));
            R.x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, ubq.re)), fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, ubq.im))};
            R.wp = A.hdt * (kh.a2s + kh.a1s);
        }
        if (t == e_ra || t == e_rb) {  // wavefront-uniform
            const double w = (t == e_ra) ? e_wa : e_wb;
            acc.re = fma(w, fma(e_wr, pr.re - p.re, p.re), acc.re);
            acc.im = fma(w, fma(e_wr, pr.im - p.im, p.im), acc.im);
        }
        return R;
    };

    // ---- prologue: rows j0-1 (halo or ghost) and j0 ----------------------
    cd hbp_m;  // hbar_Phi at row t-1
    Row cur;
    {
        cd ubp_m = {0.0, 0.0};
        if (j0 > 0) {
            const Row rm = fresh(j0 - 1, hp[0], hq[0], ubp_m, false, ang_row(j0 - 1));
            ubp_m = rm.ubp;
            hbp_m = rm.hbp;
        }
        cur = fresh(j0, hp[1], hq[1], ubp_m, true, ang_row(j0));
        if (j0 == 0) hbp_m = cscale(sg, cur.hbp);
    }
    // angular factors of the row after the next one to be finished, loaded
    // one row ahead so that their scalar loads are complete when needed
    Ang g_next = ang_row(j0 + 1);

    auto finish_row = [&](int t, cd& rp, cd& rq) {
        // row t+1: streamed, or the pole ghost row
        Row nxt;
        cd ubp_p, hbp_p;
        const Ang g1 = g_next;
        g_next = ang_row(t + 2);
        if (t + 1 < nth) {
            nxt = fresh(t + 1, rp, rq, cur.ubp, true, g1);
            ubp_p = nxt.ubp;
            hbp_p = nxt.hbp;
        } else {
            ubp_p = cscale(sg, cur.ubp);
            hbp_p = cscale(sg, cur.hbp);
            nxt = cur;  // unused: the sweep ends with this row
        }
        {
            const size_t o = (size_t)min(t + 1 + kRowsInFlight, last) * P + ci;
            rp = ld(u_in, o);
            rq = ld(u_in, o + A.plane);
        }

        // stage 1, Pi component at (i+1/2, t), and its neighbour at i-1/2
        const cd hq = {fma(cur.wp, ubp_p.re, cur.x.re), fma(cur.wp, ubp_p.im, cur.x.im)};
        const cd hql = from_left(hq);
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);

        // stage 2 at (i, t)
        //   Phi' = Phi - dt [ b dh_Phi / dr - hbar_Pi ]
        //   Pi'  = Pi  - dt [ (c dh_Phi - b dh_Pi)/dr - S_Pi(hbar) ]
        Coef ki;
        if constexpr (KERR) {
            ki = kerr_coef(Ri, cur.g, kerr_sigma(Ri, cur.g));
        } else {
            ki = user_coef(uci, nth, P, t, ci, A.inv_dth2, A.inv_2dth);
        }
        const double tb = A.dt_dr * ki.b;
        cd np = {fma(-tb, cur.dhp.re, fma(A.dt, hbq.re, cur.p.re)), fma(-tb, cur.dhp.im, fma(A.dt, hbq.im, cur.p.im))};
        const cd dq2 = d_pi(ki, cur.dhp, dhq);
        cd s2 = s_pi(ki, hbp_m, cur.hbp, hbp_p, hbq);
        if constexpr (SRC) s2 = cadd(s2, source(src_i, (size_t)t * P + ci, A.sf[2], A.sf[3]));
        cd nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, cur.q.re)), fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, cur.q.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
        }
        if (store_ok) {
            const size_t o = (size_t)t * P + col;
            st_state<KEEP>(u_out, o, np);
            st_state<KEEP>(u_out, o + A.plane, nq);
            if (win != nullptr) {  // keep the input state (for the adjoint)
                st(win, o, cur.p);
                st(win, o + A.plane, cur.q);
            }
        }

        hbp_m = cur.hbp;
        cur = nxt;
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

    if (e_id >= 0 && lane == e_lane && series != nullptr) {
        double2 w;
        w.x = acc.re;
        w.y = acc.im;
        series[e_id] = w;
    }
}

// Two Lax-Wendroff steps in one pass over a tile (temporal blocking): the
// first step's result never leaves registers.  Step A sweeps the input rows
// exactly as sweep_tile does; each row it completes, u^{n+1}(r), is fed as
// the next input row of a second sweep, step B, which completes row r-1 of
// u^{n+2}.  Per tile, A covers the rows j0-1 .. j1 that B needs (reading
// j0-2 .. j1+1) and B writes j0 .. j1-1.  Across lanes, A's results are
// valid on lanes 1..62 and B's on lanes 2..61, hence 60-column strips.
// Boundary rules are those of one step: A's radial boundary columns are
// zero before B reads them, and both sweeps use the pole ghost rows.
// Both steps need the same coefficients at the same points: B takes those A
// built one row earlier (the half-point set of row r, the integer-point set
// of row r-1) instead of rebuilding them.  The wavefront's radial factors
// live in its own LDS slice (rs: [integer/half][field][lane]), which frees
// the registers the carried coefficients need.
// Extraction is fused for both states a pass samples: the input (sample of
// step n-1) and the intermediate state (sample of step n).
typedef __attribute__((address_space(3))) double* lds_t;

template <bool KERR, bool SRC, int KEEP>
__device__ __forceinline__ void sweep_tile2(gin_t __restrict__ u_in, gout_t __restrict__ u_out, ctab_t rad,
                                            ctab_t ang, ctab_t uci, ctab_t uch, cext_t ext,
                                            double2* __restrict__ series_in, double2* __restrict__ series_mid,
                                            gout_t __restrict__ u_mid, lds_t rs, const StepScalars& A, int strip,
                                            int chunk, int lane, gin_t __restrict__ src_i = nullptr,
                                            gin_t __restrict__ src_h = nullptr) {
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols2 - 2 + lane;
    // Lanes outside the grid need no masking (as in sweep_tile): what they
    // hold reaches only the radial boundary columns of step A's and step B's
    // outputs, which both steps set to zero.
    const int ci = min(max(col, 0), nr - 1);
    const int hi = min(max(col, 0), nr - 2);

    // This lane's radial factors (kind 0: its column, kind 1: its half
    // point), loaded here and written to the wavefront's LDS slice once the
    // loads of the first rows are in flight too, so that the two latencies
    // overlap at the start of the tile.
    double tv[2 * kNumRad];
    if constexpr (KERR) {
#pragma unroll
        for (int f = 0; f < kNumRad; ++f) {
            tv[f] = rad[((size_t)f * 2 + 0) * P + ci];
            tv[kNumRad + f] = rad[((size_t)f * 2 + 1) * P + hi];
        }
    }
    // radial factors of this lane's column (kind 0) or half point (kind 1);
    // the row-dependent zero offset keeps the reads next to their use
    auto rad_lds = [&](int kind, int t) -> Rad {
        const __attribute__((address_space(3))) double* r = rs + kind * kNumRad * kWave + lane + (t & A.zero);
        Rad R;
        R.rho = r[R_RHO * kWave];
        R.rho2 = r[R_RHO2 * kWave];
        R.a2d = r[R_A2D * kWave];
        R.rb1 = r[R_RB1 * kWave];
        R.rb2 = r[R_RB2 * kWave];
        R.rb3 = r[R_RB3 * kWave];
        R.ctr = r[R_CTR * kWave];
        R.cti0 = r[R_CTI0 * kWave];
        R.cti1 = r[R_CTI1 * kWave];
        R.b1n = r[R_B1N * kWave];
        R.dl2 = r[R_DL2 * kWave];
        R.v0r = r[R_V0R * kWave];
        R.v0i = r[R_V0I * kWave];
        return R;
    };
    auto coef_h = [&](int t, const Ang& G) -> Coef {
        if constexpr (KERR) {
            const Rad R = rad_lds(1, t);
            return kerr_coef(R, G, kerr_sigma(R, G));
        } else {
            return user_coef(uch, nth, P, t, hi, A.inv_dth2, A.inv_2dth);
        }
    };
    auto coef_i = [&](int t, const Ang& G) -> Coef {
        if constexpr (KERR) {
            const Rad R = rad_lds(0, t);
            return kerr_coef(R, G, kerr_sigma(R, G));
        } else {
            return user_coef(uci, nth, P, t, ci, A.inv_dth2, A.inv_2dth);
        }
    };

    const bool store_ok = (lane >= 2) && (lane <= kWave - 3) && (col < nr);
    const bool boundary = (col == 0) || (col == nr - 1);
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const int aE = min(j1, nth - 1);         // last row step A completes
    const int lastA = min(aE + 1, nth - 1);  // last input row read
    const double sg = (double)A.sigma;

    // the (at most one) extraction point of this tile
    int e_id = -1, e_lane = 0, e_ra = -1, e_rb = -1;
    double e_wr = 0.0, e_wa = 0.0, e_wb = 0.0;
    for (int e = 0; e < A.n_ext; ++e) {
        const int ecol = ext[e].col, era = ext[e].rowa;
        const int es = ecol / kStripCols2;
        if (es == strip && era / A.rows == chunk) {
            e_id = e;
            e_lane = ecol - es * kStripCols2 + 2;
            e_ra = era;
            e_rb = ext[e].rowb;
            e_wr = ext[e].wr;
            e_wa = ext[e].wa;
            e_wb = ext[e].wb;
        }
    }
    cd acc_in = {0.0, 0.0}, acc_mid = {0.0, 0.0};
    // bilinear sample of a Phi row into acc
    auto sample = [&](int t, cd p, cd& acc) {
        if (t == e_ra || t == e_rb) {  // wavefront-uniform
            const double w = (t == e_ra) ? e_wa : e_wb;
            const cd pr = from_right(p);
            acc.re = fma(w, fma(e_wr, pr.re - p.re, p.re), acc.re);
            acc.im = fma(w, fma(e_wr, pr.im - p.im, p.im), acc.im);
        }
    };

    auto ang_row = [&](int t) -> Ang {
        Ang G{};
        if constexpr (KERR) G = load_ang(ang, nth, min(t, nth - 1));
        return G;
    };

    // Stage-1 pieces of row t (as in sweep_tile) with the half-point
    // coefficients kh of the row.  FULL = false: only the averages needed
    // from a halo row.
    // stp: the step of the pass (0: sweep A, 1: sweep B), for the source term
    auto fresh = [&](int t, cd p, cd q, cd ubp_prev, bool full, const Ang& G, const Coef& kh, int stp) -> Row {
        Row R;
        R.p = p;
        R.q = q;
        R.g = G;
        const cd pr = from_right(p), qr = from_right(q);
        R.ubp = cavg(p, pr);
        const cd ubq = cavg(q, qr);
        const cd dp = csub(pr, p);
        const double tb = A.hdt_dr * kh.b;
        const cd hp = {fma(-tb, dp.re, fma(A.hdt, ubq.re, R.ubp.re)), fma(-tb, dp.im, fma(A.hdt, ubq.im, R.ubp.im))};
        const cd hpl = from_left(hp);
        R.hbp = cavg(hp, hpl);
        R.dhp = csub(hp, hpl);
        if (full) {
            const cd dq = csub(qr, q);
            const cd um = (t == 0) ? cscale(sg, R.ubp) : ubp_prev;
            const cd dq1 = d_pi(kh, dp, dq);
            cd s1 = s_pi(kh, um, R.ubp, cd{0.0, 0.0}, ubq);
            if constexpr (SRC) s1 = cadd(s1, source(src_h, (size_t)t * P + hi, A.sf[4 * stp], A.sf[4 * stp + 1]));
            R.x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, ubq.re)), fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, ubq.im))};
            R.wp = A.hdt * (kh.a2s + kh.a1s);
        }
        return R;
    };

    // Stage 2 at (i, t) with the integer-point coefficients ki of row t: the
    // new (Phi, Pi) of row t from its stage-1 state c, hbar_Phi of row t-1
    // and (ubar_Phi, hbar_Phi) of row t+1.
    auto out_row = [&](int t, const Row& c, const Coef& ki, cd hbp_m, cd ubp_p, cd hbp_p, cd& np, cd& nq, int stp) {
        const cd hq = {fma(c.wp, ubp_p.re, c.x.re), fma(c.wp, ubp_p.im, c.x.im)};
        const cd hql = from_left(hq);
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);
        const double tb = A.dt_dr * ki.b;
        np = {fma(-tb, c.dhp.re, fma(A.dt, hbq.re, c.p.re)), fma(-tb, c.dhp.im, fma(A.dt, hbq.im, c.p.im))};
        const cd dq2 = d_pi(ki, c.dhp, dhq);
        cd s2 = s_pi(ki, hbp_m, c.hbp, hbp_p, hbq);
        if constexpr (SRC) s2 = cadd(s2, source(src_i, (size_t)t * P + ci, A.sf[4 * stp + 2], A.sf[4 * stp + 3]));
        nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, c.q.re)), fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, c.q.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
        }
    };

    // Rows are read and written through row resources (device_common.hpp):
    // lane byte offsets of the clamped column (loads) and of the owned
    // column, or none (stores).
    const int32_t row_bytes = P * (int32_t)sizeof(v2d);
    const uint32_t ld_off = (uint32_t)ci * sizeof(v2d);
    const uint32_t st_off = store_ok ? (uint32_t)col * sizeof(v2d) : kOffNone;
    auto put_row = [&](gout_t base, int t, cd vp, cd vq, auto keep) {
        const gout_t b = base + (size_t)t * P;
        st_row<decltype(keep)::value>(row_rsrc(b, row_bytes), st_off, vp);
        st_row<decltype(keep)::value>(row_rsrc(b + A.plane, row_bytes), st_off, vq);
    };

    // the intermediate state, kept for the adjoint (owned rows and columns)
    auto store_mid = [&](int t, cd vp, cd vq) {
        if (u_mid != nullptr && t >= j0 && t < j1) put_row(u_mid, t, vp, vq, std::integral_constant<int, 0>{});
    };

    auto load_row = [&](int t, cd& p, cd& q) {
        const gin_t b = u_in + (size_t)min(max(t, 0), lastA) * P;
        p = ld_row(row_rsrc(b, row_bytes), ld_off);
        q = ld_row(row_rsrc(b + A.plane, row_bytes), ld_off);
    };

    // ---- prologue: step A completes rows j0-1 (if j0 > 0) and j0; step B
    // takes them as its halo row and its first row ------------------------
    // Carried between the sweeps: kh_a = half-point coefficients of A's
    // current row (step B's next row), ki_b = integer-point coefficients of
    // the row step B completes next.
    Row a_cur, b_cur;
    Coef kh_a, ki_b;
    cd a_hbp_m, b_hbp_m;
    // The rows the prologue starts from (step A's rows aS-1 .. aS+2, i.e.
    // j0-2 .. j0+1) and the first two of the main sweep's ring, all loaded
    // before the radial factors are written to LDS.
    const int aS = max(j0 - 1, 0);
    cd pp[4], pq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_row(aS - 1 + u, pp[u], pq[u]);
    cd bp[kRowsInFlight2], bq[kRowsInFlight2];
#pragma unroll
    for (int u = 0; u < kRowsInFlight2; ++u) load_row(j0 + 2 + u, bp[u], bq[u]);
    if constexpr (KERR) {
        // this wavefront's slice: lane-private values, written and read by
        // the same lane, so no barrier is needed
#pragma unroll
        for (int f = 0; f < 2 * kNumRad; ++f) rs[f * kWave + lane] = tv[f];
    }
    {
        // step A's rows j0-2 (halo) .. j0+1
        cd ubp_m = {0.0, 0.0};
        if (aS > 0) {
            const Ang G = ang_row(aS - 1);
            const Row h = fresh(aS - 1, pp[0], pq[0], ubp_m, false, G, coef_h(aS - 1, G), 0);
            sample(aS - 1, h.p, acc_in);
            ubp_m = h.ubp;
            a_hbp_m = h.hbp;
        }
        {
            const Ang G = ang_row(aS);
            kh_a = coef_h(aS, G);
            a_cur = fresh(aS, pp[1], pq[1], ubp_m, true, G, kh_a, 0);
        }
        sample(aS, a_cur.p, acc_in);
        if (aS == 0) a_hbp_m = cscale(sg, a_cur.hbp);
        cd b_ubp_m = {0.0, 0.0};
        // A completes row r with row r+1 = (p1, q1) arriving; B takes row r
        auto prologue_row = [&](int r, cd p1, cd q1) {
            Row a_nxt;
            Coef kh_n;
            cd ubp_p, hbp_p;
            if (r + 1 < nth) {
                const Ang G = ang_row(r + 1);
                kh_n = coef_h(r + 1, G);
                a_nxt = fresh(r + 1, p1, q1, a_cur.ubp, true, G, kh_n, 0);
                sample(r + 1, a_nxt.p, acc_in);
                ubp_p = a_nxt.ubp;
                hbp_p = a_nxt.hbp;
            } else {
                ubp_p = cscale(sg, a_cur.ubp);
                hbp_p = cscale(sg, a_cur.hbp);
                a_nxt = a_cur;
                kh_n = kh_a;
            }
            ki_b = coef_i(r, a_cur.g);
            cd vp, vq;
            out_row(r, a_cur, ki_b, a_hbp_m, ubp_p, hbp_p, vp, vq, 0);
            store_mid(r, vp, vq);
            const Ang gr = a_cur.g;
            a_hbp_m = a_cur.hbp;
            a_cur = a_nxt;
            if (r < j0) {  // step B's halo row j0-1
                const Row h = fresh(r, vp, vq, b_ubp_m, false, gr, kh_a, 1);
                sample(r, h.p, acc_mid);
                b_ubp_m = h.ubp;
                b_hbp_m = h.hbp;
            } else {
                b_cur = fresh(r, vp, vq, b_ubp_m, true, gr, kh_a, 1);
                sample(r, b_cur.p, acc_mid);
                if (r == 0) b_hbp_m = cscale(sg, b_cur.hbp);
            }
            kh_a = kh_n;
        };
        prologue_row(aS, pp[2], pq[2]);                    // one or two rows,
        if (j0 > aS) prologue_row(aS + 1, pp[3], pq[3]);  // wavefront-uniform
    }

    // ---- main sweep: A completes row r (reading row r+1 from the ring), B
    // completes row r-1 --------------------------------------------------
    Ang g_next = ang_row(j0 + 2);

    // Step A completes row r (reading row r+1 from the ring), step B row
    // r-1.  The row states (A's and B's rows, the carried coefficient sets)
    // live in two copies that swap roles from row to row: ac/bc/khc/kic
    // hold row r's, the next row's arrive in an/bn/khn/kin.
    static_assert(kRowsInFlight2 == 2, "the row loop takes rows in pairs");
    // POLE: row r may be the grid's last (so may the pair loop's second row, in the last chunk)
    auto step_row = [&](int r, cd& rp, cd& rq, Row& ac, Row& an, Row& bc, Row& bn, Coef& khc, Coef& khn, Coef& kic,
                        Coef& kin, bool pole) {
        cd ubp_p, hbp_p;
        const Ang g1 = g_next;
        g_next = ang_row(r + 2);
        if (!pole || r + 1 < nth) {
            khn = coef_h(r + 1, g1);
            an = fresh(r + 1, rp, rq, ac.ubp, true, g1, khn, 0);
            sample(r + 1, an.p, acc_in);
            ubp_p = an.ubp;
            hbp_p = an.hbp;
        } else {
            ubp_p = cscale(sg, ac.ubp);
            hbp_p = cscale(sg, ac.hbp);
            an = ac;  // unused: the sweep ends with this row
            khn = khc;
        }
        load_row(r + 1 + kRowsInFlight2, rp, rq);
        kin = coef_i(r, ac.g);
        cd vp, vq;
        out_row(r, ac, kin, a_hbp_m, ubp_p, hbp_p, vp, vq, 0);
        store_mid(r, vp, vq);
        a_hbp_m = ac.hbp;

        bn = fresh(r, vp, vq, bc.ubp, true, ac.g, khc, 1);
        sample(r, bn.p, acc_mid);
        cd wp, wq;
        out_row(r - 1, bc, kic, b_hbp_m, bn.ubp, bn.hbp, wp, wq, 1);
        put_row(u_out, r - 1, wp, wq, std::integral_constant<int, KEEP>{});
        b_hbp_m = bc.hbp;
    };
    // the grid's last row: step B with the pole ghost row
    auto last_row = [&](const Row& bc, const Coef& kic) {
        cd wp, wq;
        out_row(nth - 1, bc, kic, b_hbp_m, cscale(sg, bc.ubp), cscale(sg, bc.hbp), wp, wq, 1);
        put_row(u_out, nth - 1, wp, wq, std::integral_constant<int, KEEP>{});
    };

    Row a_oth, b_oth;
    Coef kh_oth, ki_oth;
    int r0 = j0 + 1;
    // Enter the row loop as each of its iterations ends: the ring's first
    // row loaded, its second still in flight.  The compiler's waits at the
    // loop head must suit both ways in; without this they drain the ring in
    // every iteration.  (Unconditional: a wait under the loop's own guard is
    // not seen as one by the compiler.)
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(2));
    for (; r0 + 1 <= aE; r0 += 2) {
        step_row(r0, bp[0], bq[0], a_cur, a_oth, b_cur, b_oth, kh_a, kh_oth, ki_b, ki_oth, true);
        step_row(r0 + 1, bp[1], bq[1], a_oth, a_cur, b_oth, b_cur, kh_oth, kh_a, ki_oth, ki_b, true);
    }
    // at most two rows left, the last of them possibly the pole row
    if (r0 <= aE) {
        step_row(r0, bp[0], bq[0], a_cur, a_oth, b_cur, b_oth, kh_a, kh_oth, ki_b, ki_oth, true);
        if (r0 + 1 <= aE) {
            step_row(r0 + 1, bp[1], bq[1], a_oth, a_cur, b_oth, b_cur, kh_oth, kh_a, ki_oth, ki_b, true);
            if (j1 == nth) last_row(b_cur, ki_b);
        } else if (j1 == nth) {
            last_row(b_oth, ki_oth);
        }
    } else if (j1 == nth) {
        last_row(b_cur, ki_b);
    }

    if (e_id >= 0 && lane == e_lane) {
        if (series_in != nullptr) series_in[e_id] = double2{acc_in.re, acc_in.im};
        if (series_mid != nullptr) series_mid[e_id] = double2{acc_mid.re, acc_mid.im};
    }
}

// LDS for the radial factors of the two-step kernels: one slice of
// 2 x kNumRad x 64 doubles (13 KB) per wavefront, sized at launch.
constexpr size_t kRadSliceBytes = 2 * kNumRad * kWave * sizeof(double);

// SRC: the inhomogeneous variant (source profile src_i, src_h; time factors in A.sf).
template <bool KERR, bool SRC, int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4)))
    lw_step2_kernel(const double2* __restrict__ u_in, double2* __restrict__ u_out, const double* __restrict__ rad,
                    const double* __restrict__ ang, const double* __restrict__ uci, const double* __restrict__ uch,
                    const ExtPoint* __restrict__ ext, double2* __restrict__ series_in,
                    double2* __restrict__ series_mid, double2* __restrict__ u_mid, const double2* __restrict__ src_i,
                    const double2* __restrict__ src_h, StepScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int strip, chunk;
    if (A.order == kTileOrderDispatch) {
        const int tile = blockIdx.x * wpb + wave;
        strip = tile % A.n_strips;
        chunk = tile / A.n_strips;
    } else {  // XCD strips: workgroup b runs on XCD b % 8
        const int x = blockIdx.x % 8, q = (blockIdx.x / 8) * wpb + wave;
        const int s_lo = x * A.n_strips / 8, n_x = (x + 1) * A.n_strips / 8 - s_lo;
        if (n_x == 0) return;  // fewer strips than XCDs
        if (A.order == kTileOrderXcdStrip) {
            strip = s_lo + q % n_x;
            chunk = q / n_x;
        } else {
            strip = s_lo + q / A.n_chunks;
            chunk = q % A.n_chunks;
            if (strip >= s_lo + n_x) return;
        }
    }
    extern __shared__ double rad_s[];
    if (chunk >= A.n_chunks) return;  // tiles beyond the last
    sweep_tile2<KERR, SRC, KEEP>((gin_t)u_in, (gout_t)u_out, (ctab_t)rad, (ctab_t)ang, (ctab_t)uci, (ctab_t)uch,
                           (cext_t)ext, series_in, series_mid, (gout_t)u_mid,
                           (lds_t)(rad_s + (threadIdx.x / kWave) * 2 * kNumRad * kWave), A, strip, chunk, lane,
                           (gin_t)src_i, (gin_t)src_h);
}

// Small grids: k = A.bsteps steps in one launch.  A workgroup holds
// A.bcols = W + 2k consecutive columns by all ntheta rows in LDS, one point
// per thread, and takes k steps there; each step consumes one column at each
// edge (the stencil's radial reach), so after k steps its W middle columns
// hold the new state, which it writes back.  Every point's coefficients are
// built once per launch (the sweeps rebuild them every step), so a step is
// the stencil arithmetic alone, in two phases with a barrier after each:
// stage 1 (the Pi half-step of row t needs the averages of rows t -/+ 1,
// which each thread forms itself from the state) and stage 2.  The
// expressions are those of
// sweep_tile's fresh() and finish_row(), operand for operand, so the results
// equal the sweeps' bit for bit; columns outside the grid read the clamped
// edge column and, as in the sweeps, reach only the zeroed boundary columns.
// Extraction: the samples of each step's input state, in the sweeps' order.
// The points are read once per launch into LDS, each thread works out once
// which samples it takes, and the launch's series values stay in LDS until
// its last step: no global memory access inside the step loop, whose
// barriers would otherwise wait for it every step.
template <int KEEP>
__global__ void __launch_bounds__(1024)
    lw_block_kernel(const double2* __restrict__ u_in, double2* __restrict__ u_out, const double* __restrict__ rad,
                    const double* __restrict__ ang, const ExtPoint* __restrict__ ext, double2* __restrict__ series,
                    StepScalars A) {
    const int B = A.bcols, K = A.bsteps, W = B - 2 * K;
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int j = threadIdx.x % B, t = threadIdx.x / B;  // blockDim.x == B * nth
    const int c0 = blockIdx.x * W;                       // first column written
    const int col = c0 - K + j;
    const int ci = min(max(col, 0), nr - 1), hi = min(max(col, 0), nr - 2);
    const int jl = max(j - 1, 0), jr = min(j + 1, B - 1);  // neighbours (clamped at the block's edges)
    const int me = t * B + j;
    const bool boundary = (col == 0) || (col == nr - 1);
    const double sg = (double)A.sigma;
    extern __shared__ double2 lds2[];
    cd* sp = reinterpret_cast<cd*>(lds2);  // [nth][B] Phi, Pi, h_Phi, h_Pi; then 2 per point samples
    cd* sq = sp + nth * B;
    cd* sh = sq + nth * B;
    cd* shq = sh + nth * B;
    cd* se = shq + nth * B;                      // [2 per point] this step's row samples
    cd* sbuf = se + 2 * kMaxBlockExt;            // [step][point] the launch's series values
    ExtPoint* sx = reinterpret_cast<ExtPoint*>(sbuf + kMaxBlockSteps * kMaxBlockExt);  // the points

    cd p = ld(u_in, (size_t)t * P + ci), q = ld(u_in, (size_t)t * P + ci + A.plane);
    const Ang G = load_ang(ang, nth, t);
    const Rad Rh = load_rad(rad, P, 1, hi), Ri = load_rad(rad, P, 0, ci);
    const Coef kh = kerr_coef(Rh, G, kerr_sigma(Rh, G));
    const Coef ki = kerr_coef(Ri, G, kerr_sigma(Ri, G));
    sp[me] = p;
    sq[me] = q;
    if ((int)threadIdx.x < A.n_ext) sx[threadIdx.x] = ext[threadIdx.x];
    // this thread's samples: bit 2e (row a of point e) and bit 2e + 1 (row
    // b), for the points whose column the workgroup writes
    unsigned duty = 0;
    for (int e = 0; e < A.n_ext; ++e) {
        const ExtPoint E = ext[e];
        if (E.col >= c0 && E.col < c0 + W && col == E.col) {
            if (t == E.rowa) duty |= 1u << (2 * e);
            else if (t == E.rowb) duty |= 2u << (2 * e);
        }
    }
    __syncthreads();

    for (int s = 0; s < K; ++s) {
        // stage 1 at (i+1/2, t): averages, the Phi half-step and the Pi
        // half-step, with the Phi averages of rows t -/+ 1 (or the pole
        // ghost rows) formed here from the state; samples
        const cd pr = sp[t * B + jr], qr = sq[t * B + jr];
        const cd ubp = cavg(p, pr);
        const cd ubq = cavg(q, qr);
        const cd dp = csub(pr, p);
        const double tb = A.hdt_dr * kh.b;
        const cd hp = {fma(-tb, dp.re, fma(A.hdt, ubq.re, ubp.re)), fma(-tb, dp.im, fma(A.hdt, ubq.im, ubp.im))};
        const cd dq = csub(qr, q);
        sh[me] = hp;
        for (unsigned d = duty; d != 0; d &= d - 1) {
            const int b = __builtin_ctz(d);
            const double wr = sx[b >> 1].wr;
            se[b] = {fma(wr, pr.re - p.re, p.re), fma(wr, pr.im - p.im, p.im)};
        }
        const cd um = (t == 0) ? cscale(sg, ubp) : cavg(sp[me - B], sp[(t - 1) * B + jr]);
        const cd ubp_p = (t == nth - 1) ? cscale(sg, ubp) : cavg(sp[me + B], sp[(t + 1) * B + jr]);
        const cd dq1 = d_pi(kh, dp, dq);
        const cd s1 = s_pi(kh, um, ubp, cd{0.0, 0.0}, ubq);
        const cd x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, ubq.re)), fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, ubq.im))};
        const double wp = A.hdt * (kh.a2s + kh.a1s);
        const cd hq = {fma(wp, ubp_p.re, x.re), fma(wp, ubp_p.im, x.im)};
        shq[me] = hq;
        __syncthreads();

        // stage 2 at (i, t); one thread per point forms its sample
        if ((int)threadIdx.x < A.n_ext) {
            const ExtPoint E = sx[threadIdx.x];
            if (E.col >= c0 && E.col < c0 + W) {
                const cd va = se[2 * threadIdx.x];
                cd acc = {fma(E.wa, va.re, 0.0), fma(E.wa, va.im, 0.0)};
                if (E.rowb >= 0) {
                    const cd vb = se[2 * threadIdx.x + 1];
                    acc = {fma(E.wb, vb.re, acc.re), fma(E.wb, vb.im, acc.im)};
                }
                sbuf[s * kMaxBlockExt + threadIdx.x] = acc;
            }
        }
        const cd hpl = sh[t * B + jl];
        const cd hbp = cavg(hp, hpl);
        const cd dhp = csub(hp, hpl);
        const cd hbp_m = (t == 0) ? cscale(sg, hbp) : cavg(sh[me - B], sh[(t - 1) * B + jl]);
        const cd hbp_p = (t == nth - 1) ? cscale(sg, hbp) : cavg(sh[me + B], sh[(t + 1) * B + jl]);
        const cd hql = shq[t * B + jl];
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);
        const double tb2 = A.dt_dr * ki.b;
        cd np = {fma(-tb2, dhp.re, fma(A.dt, hbq.re, p.re)), fma(-tb2, dhp.im, fma(A.dt, hbq.im, p.im))};
        const cd dq2 = d_pi(ki, dhp, dhq);
        const cd s2 = s_pi(ki, hbp_m, hbp, hbp_p, hbq);
        cd nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, q.re)), fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, q.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
        }
        p = np;
        q = nq;
        sp[me] = p;
        sq[me] = q;
        __syncthreads();
    }
    if (j >= K && j < K + W && col < nr) {
        st_state<KEEP>(u_out, (size_t)t * P + col, p);
        st_state<KEEP>(u_out, (size_t)t * P + col + A.plane, q);
    }
    // the series values of the launch's steps (state row0 + s + 1 at series
    // row row0 + s; none for the initial state)
    if ((int)threadIdx.x < A.n_ext) {
        const ExtPoint E = sx[threadIdx.x];
        if (E.col >= c0 && E.col < c0 + W)
            for (int s = 0; s < K; ++s)
                if (A.row0 + s >= 0) {
                    const cd v = sbuf[s * kMaxBlockExt + threadIdx.x];
                    series[(size_t)(A.row0 + s) * A.n_ext + threadIdx.x] = double2{v.re, v.im};
                }
    }
}

__global__ void zero_ints_kernel(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <bool KERR, bool SRC, int KEEP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TEUK_WAVES_PER_SIMD, 8)))
    lw_step_kernel(const double2* __restrict__ u_in, double2* __restrict__ u_out, const double* __restrict__ rad,
                   const double* __restrict__ ang, const double* __restrict__ uci, const double* __restrict__ uch,
                   const ExtPoint* __restrict__ ext, double2* __restrict__ series, double2* __restrict__ win,
                   const double2* __restrict__ src_i, const double2* __restrict__ src_h, StepScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    // Tiles are numbered strip-fastest, so the wavefronts of a workgroup take
    // neighbouring strips of one theta chunk (their halo columns overlap).
    // Workgroups are left in dispatch order, which deals them round-robin
    // over the XCDs: measured faster for these streaming passes than giving
    // each XCD a contiguous range (whose last, short theta chunk then falls
    // on one XCD).  The tile index is made explicitly wavefront-uniform so
    // that everything derived from it (rows, table reads, loop control) is
    // scalar.
    const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x / kWave));
    const int strip = tile % A.n_strips;
    const int chunk = tile / A.n_strips;
    if (chunk >= A.n_chunks) return;  // tiles beyond the last
    sweep_tile<KERR, SRC, KEEP>((gin_t)u_in, (gout_t)u_out, (ctab_t)rad, (ctab_t)ang, (ctab_t)uci, (ctab_t)uch,
                          (cext_t)ext, series, (gout_t)win, A, strip, chunk, lane, (gin_t)src_i, (gin_t)src_h);
}

// Many grids in one persistent launch: the tiles of all members form one
// work list (member k owns tiles [tile_begin_k, tile_begin_{k+1})); each
// wavefront walks the list with a grid-wide stride.  All tiles have the
// same shape (62 columns x `rows` rows, ragged only at a member's edges),
// so the static stride balances uneven members.  `parity` selects which of
// each member's two state buffers is the input.
template <int KEEP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TEUK_WAVES_PER_SIMD, 8)))
    lw_batch_kernel(const BatchMember* __restrict__ members, int n_members, int total_tiles, int parity) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int nwaves = gridDim.x * wpb;
    const int w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x / kWave));
    for (int tile = w0; tile < total_tiles; tile += nwaves) {
        int lo = 0, hi = n_members - 1;  // last member with tile_begin <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (members[mid].tile_begin <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchMember& M = members[lo];
        const int local = tile - M.tile_begin;
        const int strip = local % M.k.n_strips;
        const int chunk = local / M.k.n_strips;
        sweep_tile<true, false, KEEP>((gin_t)M.u[parity], (gout_t)M.u[1 - parity], (ctab_t)M.rad, (ctab_t)M.ang, nullptr,
                         nullptr, nullptr, nullptr, nullptr, M.k, strip, chunk, lane);
    }
}

// The batched launch of the two-step pass: as lw_batch_kernel, over the
// members' two-step tiles.
template <int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4)))
    lw_batch2_kernel(const BatchMember* __restrict__ members, int n_members, int total_tiles, int parity) {
    extern __shared__ double rad_s[];
    const lds_t rs = (lds_t)(rad_s + (threadIdx.x / kWave) * 2 * kNumRad * kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int nwaves = gridDim.x * wpb;
    const int w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x / kWave));
    for (int tile = w0; tile < total_tiles; tile += nwaves) {
        int lo = 0, hi = n_members - 1;  // last member with tile_begin2 <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (members[mid].tile_begin2 <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchMember& M = members[lo];
        const int local = tile - M.tile_begin2;
        StepScalars k = M.k;
        k.n_strips = M.n_strips2;
        const int strip = local % k.n_strips;
        const int chunk = local / k.n_strips;
        sweep_tile2<true, false, KEEP>((gin_t)M.u[parity], (gout_t)M.u[1 - parity], (ctab_t)M.rad, (ctab_t)M.ang, nullptr,
                          nullptr, nullptr, nullptr, nullptr, nullptr, rs, k, strip, chunk, lane);
    }
}

// The state is stored as two planes in one buffer: u[f * nth * pitch + j *
// pitch + i], f = 0 for Phi and 1 for Pi.

// The row-wise kernels below take rows blockIdx.y, blockIdx.y + gridDim.y,
// ...: a launch's y dimension is capped (kMaxGridY) while ntheta may reach 2^20.
constexpr int kMaxGridY = 65535;

__global__ void import_kernel(const double2* __restrict__ src, double2* __restrict__ u, int f, int nr, int nth,
                              int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pitch) return;
    for (int j = blockIdx.y; j < nth; j += gridDim.y) {
        double2 v;
        v.x = 0.0;
        v.y = 0.0;
        if (i > 0 && i < nr - 1) v = src[(size_t)j * nr + i];
        u[(size_t)f * nth * pitch + (size_t)j * pitch + i] = v;
    }
}

__global__ void export_kernel(const double2* __restrict__ u, double2* __restrict__ dst, int f, int nr, int nth,
                              int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int j = blockIdx.y; j < nth; j += gridDim.y)
        dst[(size_t)j * nr + i] = u[(size_t)f * nth * pitch + (size_t)j * pitch + i];
}

// Bilinear sample of Phi at one extraction point (rows rowa, rowb with the
// pole ghost signs folded into the weights).
__device__ __forceinline__ double2 sample_point(const double2* __restrict__ u, int pitch, const ExtPoint& E) {
    auto row = [&](int j) {
        const double2 a = u[(size_t)j * pitch + E.col];
        const double2 b = u[(size_t)j * pitch + E.col + 1];
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
    return w;
}

__global__ void extract_kernel(const double2* __restrict__ u, int pitch, const ExtPoint* __restrict__ pts, int n,
                               double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    out[e] = sample_point(u, pitch, pts[e]);
}

// Psi(t_k, observer o) = sum over modes j of e^{i m_j phi_o} r_o^3 Phi_{m_j}(t_k, o)
// (the field from its azimuthal modes, Sec. 3.2); samples are
// [n_samples][n_modes][n_obs], psi [n_samples][n_obs].  The modes are summed
// in their given order.
__global__ void assemble_kernel(AssembleArgs A, int64_t n_samples, const double2* __restrict__ samples,
                                double2* __restrict__ psi) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_samples * A.n_obs) return;
    const int64_t k = id / A.n_obs;
    const int o = (int)(id % A.n_obs);
    double re = 0.0, im = 0.0;
    for (int j = 0; j < A.n_modes; ++j) {
        double sn, cs;
        sincos(A.m[j] * A.phi[o], &sn, &cs);
        const double2 f = samples[(k * A.n_modes + j) * A.n_obs + o];
        re = fma(cs, f.x, fma(-sn, f.y, re));
        im = fma(cs, f.y, fma(sn, f.x, im));
    }
    psi[id] = double2{A.r3[o] * re, A.r3[o] * im};
}

// Samples of every member's extraction points of a batch, in member order.
__global__ void batch_extract_kernel(const BatchExtPoint* __restrict__ pts, int n, int parity,
                                     double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const BatchExtPoint& P = pts[e];
    out[e] = sample_point(P.u[parity], P.pitch, P.e);
}

__global__ void nonfinite_kernel(const double2* __restrict__ u, int nr, int nth, int pitch, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int j = blockIdx.y; j < nth; j += gridDim.y) {
        const size_t o = (size_t)j * pitch + i;
        const double2 a = u[o], b = u[o + (size_t)nth * pitch];
        if (!isfinite(a.x) || !isfinite(a.y) || !isfinite(b.x) || !isfinite(b.y)) *flag = 1;
    }
}

// As nonfinite_kernel for the in-loop check: the first check (in stream
// order) that finds a non-finite value records its step count (>= 1).
__global__ void nonfinite_step_kernel(const double2* __restrict__ u, int nr, int nth, int pitch,
                                      unsigned long long* first, long long step) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    bool bad = false;
    for (int j = blockIdx.y; j < nth; j += gridDim.y) {
        const size_t o = (size_t)j * pitch + i;
        const double2 a = u[o], b = u[o + (size_t)nth * pitch];
        bad = bad || !isfinite(a.x) || !isfinite(a.y) || !isfinite(b.x) || !isfinite(b.y);
    }
    if (bad) atomicCAS(first, 0ull, (unsigned long long)step);
}

__global__ void pitch_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int rows, int cols,
                                  int pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pitch) return;
    for (int j = blockIdx.y; j < rows; j += gridDim.y)
        dst[(size_t)j * pitch + i] = (i < cols) ? src[(size_t)j * cols + i] : 0.0;
}

}  // namespace

hipError_t launch_step(const StepArgs& a, bool kerr, int waves_per_block, hipStream_t s) {
    const int nb = (a.k.n_strips * a.k.n_chunks + waves_per_block - 1) / waves_per_block;
    const dim3 block(kWave * waves_per_block), grid(nb);
    const bool src = a.src_i != nullptr;
    const int keep = a.k.keep ? 1 : 0;
    auto pick = [&](auto k0, auto k1) { return keep ? k1 : k0; };
    auto kern = kerr ? (src ? pick(lw_step_kernel<true, true, 0>, lw_step_kernel<true, true, 1>)
                            : pick(lw_step_kernel<true, false, 0>, lw_step_kernel<true, false, 1>))
                     : (src ? pick(lw_step_kernel<false, true, 0>, lw_step_kernel<false, true, 1>)
                            : pick(lw_step_kernel<false, false, 0>, lw_step_kernel<false, false, 1>));
    hipLaunchKernelGGL(kern, grid, block, 0, s, a.u_in, a.u_out, a.rad, a.ang, a.uci, a.uch,
                       a.ext, a.series, a.win, a.src_i, a.src_h, a.k);
    return hipGetLastError();
}

hipError_t launch_block(const StepArgs& a, hipStream_t s) {
    const int w = a.k.bcols - 2 * a.k.bsteps;
    const dim3 grid((a.k.nr + w - 1) / w), block(a.k.bcols * a.k.nth);
    static_assert(sizeof(ExtPoint) == 3 * sizeof(double2), "the points' LDS area");
    if (a.k.bsteps > kMaxBlockSteps || a.k.n_ext > kMaxBlockExt) return hipErrorInvalidValue;
    const size_t lds =
        (size_t)(4 * a.k.nth * a.k.bcols + 2 * kMaxBlockExt + kMaxBlockSteps * kMaxBlockExt + 3 * kMaxBlockExt) *
        sizeof(double2);
    hipLaunchKernelGGL(a.k.keep ? lw_block_kernel<1> : lw_block_kernel<0>, grid, block, lds, s, a.u_in, a.u_out,
                       a.rad, a.ang, a.ext, a.series, a.k);
    return hipGetLastError();
}

hipError_t launch_step2(const StepArgs& a, bool kerr, int waves_per_block, hipStream_t s) {
    // XCD orders: 8 equal shares of workgroups, each covering the tiles of
    // the largest XCD run of strips
    const int per_xcd = (a.k.n_strips + 7) / 8 * a.k.n_chunks;
    const int nb = a.k.order == kTileOrderDispatch
                       ? (a.k.n_strips * a.k.n_chunks + waves_per_block - 1) / waves_per_block
                       : 8 * ((per_xcd + waves_per_block - 1) / waves_per_block);
    const dim3 block(kWave * waves_per_block), grid(nb);
    const bool src = a.src_i != nullptr;
    const int keep = a.k.keep ? 1 : 0;
    auto pick = [&](auto k0, auto k1) { return keep ? k1 : k0; };
    auto kern = kerr ? (src ? pick(lw_step2_kernel<true, true, 0>, lw_step2_kernel<true, true, 1>)
                            : pick(lw_step2_kernel<true, false, 0>, lw_step2_kernel<true, false, 1>))
                     : (src ? pick(lw_step2_kernel<false, true, 0>, lw_step2_kernel<false, true, 1>)
                            : pick(lw_step2_kernel<false, false, 0>, lw_step2_kernel<false, false, 1>));
    hipLaunchKernelGGL(kern, grid, block, kerr ? waves_per_block * kRadSliceBytes : 0, s, a.u_in, a.u_out, a.rad, a.ang,
                       a.uci, a.uch, a.ext, a.series, a.series_mid, a.win, a.src_i, a.src_h, a.k);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchMember* members, int n_members, int total_tiles, int parity, int n_blocks,
                        int waves_per_block, bool two, bool keep, hipStream_t s) {
    if (two) {
        const int w = waves_per_block < 4 ? waves_per_block : 4;
        hipLaunchKernelGGL(keep ? lw_batch2_kernel<1> : lw_batch2_kernel<0>, dim3(n_blocks), dim3(kWave * w),
                           w * kRadSliceBytes, s, members, n_members, total_tiles, parity);
    } else {
        hipLaunchKernelGGL(keep ? lw_batch_kernel<1> : lw_batch_kernel<0>, dim3(n_blocks),
                           dim3(kWave * waves_per_block), 0, s, members, n_members, total_tiles, parity);
    }
    return hipGetLastError();
}

hipError_t launch_import(const double2* src, double2* u, int f, int nr, int nth, int pitch, hipStream_t s) {
    const dim3 block(256), grid((pitch + 255) / 256, std::min(nth, kMaxGridY));
    hipLaunchKernelGGL(import_kernel, grid, block, 0, s, src, u, f, nr, nth, pitch);
    return hipGetLastError();
}

hipError_t launch_export(const double2* u, double2* dst, int f, int nr, int nth, int pitch, hipStream_t s) {
    const dim3 block(256), grid((nr + 255) / 256, std::min(nth, kMaxGridY));
    hipLaunchKernelGGL(export_kernel, grid, block, 0, s, u, dst, f, nr, nth, pitch);
    return hipGetLastError();
}

hipError_t launch_extract(const double2* u, int pitch, const ExtPoint* pts, int n, double2* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 block(64), grid((n + 63) / 64);
    hipLaunchKernelGGL(extract_kernel, grid, block, 0, s, u, pitch, pts, n, out);
    return hipGetLastError();
}

hipError_t launch_batch_extract(const BatchExtPoint* pts, int n, int parity, double2* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 block(64), grid((n + 63) / 64);
    hipLaunchKernelGGL(batch_extract_kernel, grid, block, 0, s, pts, n, parity, out);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs& a, int64_t n_samples, const double2* samples, double2* psi,
                           hipStream_t s) {
    const int64_t n = n_samples * a.n_obs;
    if (n <= 0) return hipSuccess;
    const dim3 block(256), grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(assemble_kernel, grid, block, 0, s, a, n_samples, samples, psi);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const double2* u, int nr, int nth, int pitch, int* flag, hipStream_t s) {
    const dim3 block(256), grid((nr + 255) / 256, std::min(nth, kMaxGridY));
    hipLaunchKernelGGL(nonfinite_kernel, grid, block, 0, s, u, nr, nth, pitch, flag);
    return hipGetLastError();
}

hipError_t launch_nonfinite_step(const double2* u, int nr, int nth, int pitch, long long* first, int64_t step,
                                 hipStream_t s) {
    const dim3 block(256), grid((nr + 255) / 256, std::min(nth, kMaxGridY));
    hipLaunchKernelGGL(nonfinite_step_kernel, grid, block, 0, s, u, nr, nth, pitch,
                       reinterpret_cast<unsigned long long*>(first), (long long)step);
    return hipGetLastError();
}

hipError_t launch_pitch_copy(const double* src, double* dst, int rows, int cols, int pitch, hipStream_t s) {
    const dim3 block(256), grid((pitch + 255) / 256, std::min(rows, kMaxGridY));
    hipLaunchKernelGGL(pitch_copy_kernel, grid, block, 0, s, src, dst, rows, cols, pitch);
    return hipGetLastError();
}

}  // namespace teuk
