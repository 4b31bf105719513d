// gfx950 adjoint of the Lax-Wendroff step (arXiv:1010.3816, Eqs. (lw1)-(lw2)
// with the boundary conditions): lambda^m = A^H lambda^{m+1} and the spin
// gradient contribution Re <lambda^{m+1}, (dA/da) u^m>.
//
// The step is complex-linear, so its adjoint for a real loss (gradient
// convention dL/dRe + i dL/dIm) is the conjugate transpose.  The kernel is
// the gather form of the transposed step and sweeps the same tiles as the
// forward kernel (64 r* columns per wavefront, theta rows in order):
//   * stage 2 transposed at integer points: nu = lambda^{m+1} with the
//     radial boundary columns zeroed gives the cotangents of hbar and dh;
//     the theta stencil of S becomes a stencil over the cotangents of rows
//     t-1, t, t+1 (each row emits an "up", "mid" and "down" part);
//   * hbar/dh transposed to the half points: lane L adds lane L+1's share;
//   * stage 1 transposed at half points, again with a row stencil;
//   * averaging/difference transposed back to integer points: lane L adds
//     lane L-1's share; plus the direct term nu.
// The spin gradient needs the forward intermediates of step m (ubar, delta,
// hbar, dh), which are recomputed from u^m exactly as in the forward
// kernel, and the a-derivatives of the coefficients, obtained by forward
// differentiation of their reconstruction from the radial tables and their
// a-derivative tables (held in LDS for the workgroup's strip).
#include "adjoint_common.hpp"

namespace teuk {
namespace {


// d/da of kerr_coef at one position from the a-derivative tables rd, four
// value fields (rv), the angular factors, s = (1/Sigma, 1/Sigma^2) and the
// coefficient values c.  With w = d(Sigma^2)/Sigma^2, a coefficient
// X/Sigma^2 has derivative dX/Sigma^2 - c w and rho/Sigma has
// drho/Sigma - c w/2, so most value fields are not needed again.
__device__ __forceinline__ Coef kerr_coef_da(lds_cptr rv, lds_cptr rd, int o, const Ang& G, Sig s, const Coef& c) {
    auto d = [&](int f) { return rd[o + f * kWave]; };
    auto v = [&](int f) { return rv[o + f * kWave]; };
    const double w = s.inv * fma(-d(R_A2D), G.sn2, d(R_RHO2));
    const double hw = 0.5 * w;
    Coef r;
    r.b = fma(s.isig, d(R_RHO), -c.b * hw);
    const double T = fma(-v(R_RB3), G.sn2, v(R_RB2));
    const double dT = fma(-d(R_RB3), G.sn2, d(R_RB2));
    const double Q = fma(-T, s.inv, v(R_RB1));
    const double dQ = fma(-s.inv, fma(-T, w, dT), d(R_RB1));
    const double bp = s.isig * Q;
    const double dbp = s.isig * fma(-Q, hw, dQ);
    r.ctr = fma(s.inv, d(R_CTR), -c.ctr * w);
    r.cti = fma(s.inv, fma(d(R_CTI1), G.cs, d(R_CTI0)), -c.cti * w);
    const double b1 = v(R_B1N) * s.inv;
    const double db1 = fma(s.inv, d(R_B1N), -b1 * w);
    r.cre = fma(r.b, bp - c.ctr, c.b * (dbp - r.ctr)) - db1;
    r.cim = -fma(r.b, c.cti, c.b * r.cti);
    r.a2s = fma(s.inv, d(R_DL2), -c.a2s * w);
    r.a1s = r.a2s * G.cotp;
    r.v0r = fma(s.inv, fma(d(R_DL2), G.pd, d(R_V0R)), -c.v0r * w);
    r.v0i = fma(s.inv, d(R_V0I), -c.v0i * w);
    return r;
}



// Extraction points (of the first n) whose bilinear stencil touches output
// rows r_lo .. r_hi of a tile and the columns c0 .. c0 + 63 of its lanes, as
// bits: the transposed extraction is applied row by row only for these.
__device__ __forceinline__ unsigned ext_mask(const ExtPoint* __restrict__ ext, int n, int r_lo, int r_hi, int c0) {
    unsigned m = 0;
    for (int e = 0; e < n; ++e) {
        const ExtPoint E = ext[e];
        const bool rows = (E.rowa >= r_lo && E.rowa <= r_hi) || (E.rowb >= r_lo && E.rowb <= r_hi);
        if (rows && E.col + 1 >= c0 && E.col <= c0 + kWave - 1) m |= 1u << e;
    }
    return m;
}

// complex helpers for the transposed operators
__device__ __forceinline__ cd cadd3(cd a, cd b, cd c) { return {a.re + b.re + c.re, a.im + b.im + c.im}; }
// (x + i y) * (re + i im)
__device__ __forceinline__ cd cmul(double x, double y, cd v) {
    return {fma(x, v.re, -y * v.im), fma(x, v.im, y * v.re)};
}

// Rows of input loaded ahead of the row being finished.  One keeps the
// kernel within the registers of two wavefronts per SIMD.
#ifndef TEUK_ADJ_ROWS_IN_FLIGHT
#define TEUK_ADJ_ROWS_IN_FLIGHT 1
#endif
constexpr int kAdjRowsInFlight = TEUK_ADJ_ROWS_IN_FLIGHT;
// The cotangent-only kernel holds far fewer values per row.
#ifndef TEUK_ADJ_ROWS_IN_FLIGHT_NOSPIN
#define TEUK_ADJ_ROWS_IN_FLIGHT_NOSPIN 2
#endif
static_assert(TEUK_ADJ_ROWS_IN_FLIGHT == 1 || TEUK_ADJ_ROWS_IN_FLIGHT == 2, "the row loop takes rows in pairs");
static_assert(TEUK_ADJ_ROWS_IN_FLIGHT_NOSPIN == 1 || TEUK_ADJ_ROWS_IN_FLIGHT_NOSPIN == 2,
              "the row loop takes rows in pairs");

// Per-row state carried from the row's arrival to its completion.  The
// forward recompute is needed for the spin gradient only.
template <bool SPIN>
struct AdjFwd {
    cd ubp, ubq, dp, dq;  // half point i+1/2
    cd hbp, dhp;          // integer point i
    cd x;                 // stage-1 Pi value at the half, minus its row-(t+1) term
    double wp;
};
template <>
struct AdjFwd<false> {};

// Tangent rows of the spin gradient's dot product (DOT kernels only).
template <bool DOT>
struct AdjTan {
    cd tp, tq;            // T_m = (dA/da) u^m at (i, t)
};
template <>
struct AdjTan<false> {};

template <bool SPIN, bool DOT = false>
struct AdjRow {
    AdjFwd<SPIN> f;       // forward recompute of step m at this row
    AdjTan<DOT> tan;      // tangent row, for the dot product with nu
    // adjoint
    cd np, nq;            // nu at (i, t), radial boundary columns zeroed
    cd lhq;               // cotangent of the stage-1 Pi value at the half
    cd up, dn;            // stage-2 theta-stencil pieces to rows t+1, t-1
    cd uph, dnh;          // stage-1 theta-stencil pieces to rows t+1, t-1
    Sig si, sh;           // 1/Sigma, 1/Sigma^2 at the integer and half point
    Ang g;                // angular factors of the row (wavefront-uniform)
};

// SPIN = false: the cotangents only.  The step is linear in the state, so
// they do not need u^m: no state rows are read, nothing of the forward step
// is recomputed and no spin gradient is accumulated.
// DOT (with SPIN = false): u_in holds T_m = (dA/da) u^m (lw_tangent_kernel)
// instead of u^m, and the spin gradient's term of this step is the dot
// product Re <lambda^{m+1}, T_m> over the owned points.
template <bool SPIN, bool DOT, int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    lw_adjoint_kernel(const double2* __restrict__ nu_in, const double2* __restrict__ u_in,
                      double2* __restrict__ lam_out, const double* __restrict__ rad,
                      const double* __restrict__ rad_da, const double* __restrict__ ang,
                      double* __restrict__ dlda_slots, const ExtPoint* __restrict__ ext,
                      const double* __restrict__ gsample, AdjScalars A) {
    constexpr int kRIF = SPIN ? kAdjRowsInFlight : TEUK_ADJ_ROWS_IN_FLIGHT_NOSPIN;
    static_assert(!(SPIN && DOT), "the stored-tangent dot product replaces the spin recompute");
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const TileOf T = tile_of(xcd_block(blockIdx.x, gridDim.x), wpb, wave, A.n_strips, A.n_chunks);
    const int strip = T.strip, chunk = T.chunk;
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols - 1 + lane;
    const unsigned long long interior = ((col >= 1) && (col < nr - 1)) ? ~0ull : 0ull;
    const int ci = min(max(col, 0), nr - 1);

    // the radial tables of the workgroup's strips: [strip][value/derivative][integer/half][field][lane]
    // (dynamic LDS, adjoint_lds_bytes)
    constexpr int kF = (SPIN ? 4 : 2) * kNumRad;
    extern __shared__ double rad_s[];
    for (int f = wave; f < T.n_slices * kF; f += wpb) {
        const int g = f % kF, deriv = g / (2 * kNumRad), kind = (g / kNumRad) % 2, field = g % kNumRad;
        const int c = min(max((T.s0 + f / kF) * kStripCols - 1 + lane, 0), nr - 1);
        const double* src = deriv ? rad_da : rad;
        rad_s[f * kWave + lane] = src[((size_t)field * 2 + kind) * P + (kind == 0 ? c : min(c, nr - 2))];
    }
    __syncthreads();
    if (!T.valid) return;  // wavefront-uniform
    const double* slice = rad_s + T.slice * kF * kWave + lane;
    lds_cptr rvi = (lds_cptr)(slice + 0 * kNumRad * kWave);
    lds_cptr rvh = (lds_cptr)(slice + 1 * kNumRad * kWave);
    lds_cptr rdi = (lds_cptr)(slice + 2 * kNumRad * kWave);
    lds_cptr rdh = (lds_cptr)(slice + 3 * kNumRad * kWave);

    const bool own = (lane >= 1) && (lane <= kWave - 2) && (col < nr);  // columns and halves this tile owns
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const double sg = (double)A.sigma;
    const int last = (j1 < nth) ? j1 : nth - 1;
    double acc = 0.0;  // spin-gradient partial sum of this lane
    const unsigned emask = ext_mask(ext, gsample ? A.n_ext : 0, j0, j1 - 1, strip * kStripCols - 1);

    // angular factors of row t (clamped: rows past the last are loaded
    // ahead but never used)
    auto ang_row = [&](int t) -> Ang { return load_ang(ang, nth, min(t, nth - 1)); };
    auto coefs = [&](int t, const Ang& G, Coef& ki, Coef& kh, Sig& si, Sig& sh) {
        const int o = t & A.zero;
        const Rad Ri = rad_from_lds(rvi, o), Rh = rad_from_lds(rvh, o);
        si = kerr_sigma(Ri, G);
        sh = kerr_sigma(Rh, G);
        ki = kerr_coef(Ri, G, si);
        kh = kerr_coef(Rh, G, sh);
    };

    // Arrival of row t: forward stage-1 pieces of u^m and the same-row part
    // of the transposed step applied to nu.
    auto fresh = [&](int t, cd p, cd q, cd np, cd nq, cd ubp_prev, const Ang& G) -> AdjRow<SPIN, DOT> {
        AdjRow<SPIN, DOT> R;
        if constexpr (DOT) {
            R.tan.tp = p;
            R.tan.tq = q;
        }
        Coef ki, kh;
        Sig si, sh;
        coefs(t, G, ki, kh, si, sh);
        R.si = si;
        R.sh = sh;
        R.g = G;
        if constexpr (SPIN) {  // forward (as in the step kernel)
            // Lanes outside the grid hold the clamped edge column, unmasked:
            // a spin term of an owned column reads them only at the radial
            // boundary, multiplied by cotangents that are zero there.
            AdjFwd<true>& F = R.f;
            const cd pr = from_right(p), qr = from_right(q);
            F.ubp = cavg(p, pr);
            F.ubq = cavg(q, qr);
            F.dp = csub(pr, p);
            F.dq = csub(qr, q);
            const double tb = A.hdt_dr * kh.b;
            const cd hp = {fma(-tb, F.dp.re, fma(A.hdt, F.ubq.re, F.ubp.re)),
                           fma(-tb, F.dp.im, fma(A.hdt, F.ubq.im, F.ubp.im))};
            const cd hpl = from_left(hp);
            F.hbp = cavg(hp, hpl);
            F.dhp = csub(hp, hpl);
            const cd um = (t == 0) ? cscale(sg, F.ubp) : ubp_prev;
            const cd dq1 = d_pi(kh, F.dp, F.dq);
            const cd s1 = s_pi(kh, um, F.ubp, cd{0.0, 0.0}, F.ubq);
            F.x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, F.ubq.re)),
                   fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, F.ubq.im))};
            F.wp = A.hdt * (kh.a2s + kh.a1s);
        }
        // adjoint, stage 2 at (i, t):
        //   Phi' = Phi + dt hbar_Pi - dt/dr b dh_Phi
        //   Pi'  = Pi - dt/dr (c dh_Phi - b dh_Pi) + dt S_Pi(hbar)
        R.np = masked(np, interior);
        R.nq = masked(nq, interior);
        const cd sq = cscale(A.dt, R.nq);                                   // cotangent of S_Pi(hbar)
        R.up = cscale(ki.a2s + ki.a1s, sq);
        R.dn = cscale(ki.a2s - ki.a1s, sq);
        const cd lhbq = cadd(cscale(A.dt, R.np), cmul(-ki.ctr, ki.cti, sq));  // + conj(-Ct) sq
        const cd ldhq = cscale(A.dt_dr * ki.b, R.nq);
        // hbar/dh -> half point i+1/2: own (1/2 hbar + dh) + right neighbour's (1/2 hbar - dh)
        const cd aq = {fma(0.5, lhbq.re, ldhq.re), fma(0.5, lhbq.im, ldhq.im)};
        const cd bq = {fma(0.5, lhbq.re, -ldhq.re), fma(0.5, lhbq.im, -ldhq.im)};
        R.lhq = cadd(aq, from_right(bq));
        // stage 1 at (i+1/2, t): h_Pi = ubar_Pi - dt/2dr (c delta_Phi - b delta_Pi) + dt/2 S_Pi(ubar)
        const cd tq = cscale(A.hdt, R.lhq);
        R.uph = cscale(kh.a2s + kh.a1s, tq);
        R.dnh = cscale(kh.a2s - kh.a1s, tq);
        return R;
    };

    // rows of u^m (or T_m) are read only for the spin gradient
    auto ldu = [&](size_t o) -> cd {
        if constexpr (SPIN || DOT) return ld(u_in, o);
        return cd{0.0, 0.0};
    };

    // ---- prologue ----------------------------------------------------------
    AdjRow<SPIN, DOT> cur;
    cd ubp_m, hbp_m, below, below_h;
    {
        cd ubp_prev = {0.0, 0.0};
        if (j0 > 0) {
            const size_t o = (size_t)(j0 - 1) * P + ci;
            const AdjRow<SPIN, DOT> rm = fresh(j0 - 1, ldu(o), ldu(o + A.plane), ld(nu_in, o), ld(nu_in, o + A.plane),
                                          ubp_prev, ang_row(j0 - 1));
            if constexpr (SPIN) {
                ubp_prev = rm.f.ubp;
                ubp_m = rm.f.ubp;
                hbp_m = rm.f.hbp;
            }
            below = rm.up;
            below_h = rm.uph;
        }
        const size_t o = (size_t)j0 * P + ci;
        cur = fresh(j0, ldu(o), ldu(o + A.plane), ld(nu_in, o), ld(nu_in, o + A.plane), ubp_prev, ang_row(j0));
        if (j0 == 0) {
            if constexpr (SPIN) {
                ubp_m = cscale(sg, cur.f.ubp);
                hbp_m = cscale(sg, cur.f.hbp);
            }
            below = cscale(sg, cur.dn);
            below_h = cscale(sg, cur.dnh);
        }
    }
    Ang g_next = ang_row(j0 + 1);  // angular factors one row ahead
    cd bu[kRIF][2], bn[kRIF][2];
#pragma unroll
    for (int k = 0; k < kRIF; ++k) {
        const size_t o = (size_t)min(j0 + 1 + k, last) * P + ci;
        bu[k][0] = ldu(o);
        bu[k][1] = ldu(o + A.plane);
        bn[k][0] = ld(nu_in, o);
        bn[k][1] = ld(nu_in, o + A.plane);
    }

    // Row t is in cur; row t+1 arrives into nxt (the two alternate roles
    // from row to row, so no row state is copied).
    auto finish_row = [&](int t, AdjRow<SPIN, DOT>& cur, AdjRow<SPIN, DOT>& nxt, cd* ru, cd* rn) {
        cd ubp_p, hbp_p, above, above_h;
        const Ang g1 = g_next;
        g_next = ang_row(t + 2);
        if (t + 1 < nth) {
            cd ubp_cur = {0.0, 0.0};
            if constexpr (SPIN) ubp_cur = cur.f.ubp;
            nxt = fresh(t + 1, ru[0], ru[1], rn[0], rn[1], ubp_cur, g1);
            if constexpr (SPIN) {
                ubp_p = nxt.f.ubp;
                hbp_p = nxt.f.hbp;
            }
            above = nxt.dn;
            above_h = nxt.dnh;
        } else {
            if constexpr (SPIN) {
                ubp_p = cscale(sg, cur.f.ubp);
                hbp_p = cscale(sg, cur.f.hbp);
            }
            above = cscale(sg, cur.up);
            above_h = cscale(sg, cur.uph);
            nxt = cur;  // unused: the sweep ends with this row
        }
        {
            const size_t o = (size_t)min(t + 1 + kRIF, last) * P + ci;
            ru[0] = ldu(o);
            ru[1] = ldu(o + A.plane);
            rn[0] = ld(nu_in, o);
            rn[1] = ld(nu_in, o + A.plane);
        }
        // coefficients of row t again (rebuilding them from the tables is
        // cheaper than keeping them in registers since the row arrived)
        const Ang& G = cur.g;
        const Sig si = cur.si, sh = cur.sh;
        Coef ki, kh;
        {
            const int o = t & A.zero;
            ki = kerr_coef(rad_from_lds(rvi, o), G, si);
            kh = kerr_coef(rad_from_lds(rvh, o), G, sh);
        }

        // adjoint: hbar_Phi cotangent complete, then stage 1 transposed at the half
        // the row's own stage-2 theta piece and dh_Phi cotangent (rebuilt
        // here rather than kept in registers since the row arrived)
        const cd mid = cmul(-2.0 * ki.a2s - ki.v0r, ki.v0i, cscale(A.dt, cur.nq));  // (-2 A2 - conj V0) sq
        const cd cnq = cmul(ki.cre, -ki.cim, cur.nq);                                // conj(c) nq
        const cd ldhp = {-A.dt_dr * fma(ki.b, cur.np.re, cnq.re), -A.dt_dr * fma(ki.b, cur.np.im, cnq.im)};
        const cd lhbp = cadd3(mid, below, above);
        const cd ap = {fma(0.5, lhbp.re, ldhp.re), fma(0.5, lhbp.im, ldhp.im)};
        const cd bp = {fma(0.5, lhbp.re, -ldhp.re), fma(0.5, lhbp.im, -ldhp.im)};
        const cd lhp = cadd(ap, from_right(bp));
        //   h_Phi = ubar_Phi + dt/2 ubar_Pi - dt/2dr b delta_Phi
        const cd midh = cmul(-2.0 * kh.a2s - kh.v0r, kh.v0i, cscale(A.hdt, cur.lhq));
        const cd lubp = cadd(lhp, cadd3(midh, below_h, above_h));
        const cd ctq = cmul(-kh.ctr, kh.cti, cur.lhq);                      // conj(-Ct) lhq
        const cd lubq = {fma(A.hdt, lhp.re, fma(A.hdt, ctq.re, cur.lhq.re)),
                         fma(A.hdt, lhp.im, fma(A.hdt, ctq.im, cur.lhq.im))};
        const cd cq = cmul(kh.cre, -kh.cim, cur.lhq);                        // conj(c) lhq
        const cd ldp = {-A.hdt_dr * fma(kh.b, lhp.re, cq.re), -A.hdt_dr * fma(kh.b, lhp.im, cq.im)};
        const cd ldq = cscale(A.hdt_dr * kh.b, cur.lhq);
        // ubar/delta -> integer points: own (1/2 ubar - delta) + left neighbour's (1/2 ubar + delta)
        const cd cP = {fma(0.5, lubp.re, ldp.re), fma(0.5, lubp.im, ldp.im)};
        const cd cQ = {fma(0.5, lubq.re, ldq.re), fma(0.5, lubq.im, ldq.im)};
        const cd dP = {fma(0.5, lubp.re, -ldp.re), fma(0.5, lubp.im, -ldp.im)};
        const cd dQ = {fma(0.5, lubq.re, -ldq.re), fma(0.5, lubq.im, -ldq.im)};
        cd outp = cadd3(cur.np, dP, from_left(cP));
        const cd outq = cadd3(cur.nq, dQ, from_left(cQ));
        // transposed extraction of the sample of the output state: each
        // stencil point of an extraction point receives its bilinear weight
        // times the sample's gradient (gsample[e], re/im interleaved)
        if (emask != 0) {
            for (int e = 0; e < A.n_ext; ++e) {
                if (!((emask >> e) & 1u)) continue;
                const ExtPoint E = ext[e];
                if (t != E.rowa && t != E.rowb) continue;  // wavefront-uniform
                const double wrow = (t == E.rowa) ? E.wa : E.wb;
                const double w = (col == E.col) ? wrow * (1.0 - E.wr) : (col == E.col + 1) ? wrow * E.wr : 0.0;
                outp.re = fma(w, gsample[2 * e], outp.re);
                outp.im = fma(w, gsample[2 * e + 1], outp.im);
            }
        }
        if (own) {
            const size_t o = (size_t)t * P + col;
            st_state<KEEP>(lam_out, o, outp);
            st_state<KEEP>(lam_out, o + A.plane, outq);
        }

        // spin gradient: coefficient derivatives against the cotangents of
        // the stage outputs, at the owned half point and integer point
        if constexpr (SPIN) {
            // forward stage-1 Pi value at the halves i+1/2, i-1/2 of row t
            const AdjFwd<true>& F = cur.f;
            const cd hq = {fma(F.wp, ubp_p.re, F.x.re), fma(F.wp, ubp_p.im, F.x.im)};
            const cd hql = from_left(hq);
            const cd hbq = cavg(hq, hql);
            const cd dhq = csub(hq, hql);
            const int o = t & A.zero;
            const Coef dkh = kerr_coef_da(rvh, rdh, o, G, sh, kh);
            const Coef dki = kerr_coef_da(rvi, rdi, o, G, si, ki);
            // half: dh_Phi = -dt/2dr db delta_Phi;  dh_Pi = -dt/2dr (dc dP - db dQ) + dt/2 dS(ubar)
            const cd dhP = cscale(-A.hdt_dr * dkh.b, F.dp);
            const cd dd1 = d_pi(dkh, F.dp, F.dq);
            const cd ds1 = s_pi(dkh, ubp_m, F.ubp, ubp_p, F.ubq);
            const cd dhQ = {fma(A.hdt, ds1.re, -A.hdt_dr * dd1.re), fma(A.hdt, ds1.im, -A.hdt_dr * dd1.im)};
            // integer: dPhi' = -dt/dr db dh_Phi;  dPi' = -dt/dr (dc dhP - db dhQ) + dt dS(hbar)
            const cd dPp = cscale(-A.dt_dr * dki.b, F.dhp);
            const cd dd2 = d_pi(dki, F.dhp, dhq);
            const cd ds2 = s_pi(dki, hbp_m, F.hbp, hbp_p, hbq);
            const cd dQp = {fma(A.dt, ds2.re, -A.dt_dr * dd2.re), fma(A.dt, ds2.im, -A.dt_dr * dd2.im)};
            double c = lhp.re * dhP.re + lhp.im * dhP.im;
            c = fma(cur.lhq.re, dhQ.re, fma(cur.lhq.im, dhQ.im, c));
            c = fma(cur.np.re, dPp.re, fma(cur.np.im, dPp.im, c));
            c = fma(cur.nq.re, dQp.re, fma(cur.nq.im, dQp.im, c));
            if (own) acc += c;
        }

        // spin gradient from the stored tangent: Re <nu, T_m> (T_m is zero on
        // the radial boundary columns, where nu is masked)
        if constexpr (DOT) {
            double c = cur.np.re * cur.tan.tp.re + cur.np.im * cur.tan.tp.im;
            c = fma(cur.nq.re, cur.tan.tq.re, fma(cur.nq.im, cur.tan.tq.im, c));
            if (own) acc += c;
        }

        below = cur.up;
        below_h = cur.uph;
        if constexpr (SPIN) {
            ubp_m = cur.f.ubp;
            hbp_m = cur.f.hbp;
        }
    };

    // rows in pairs (the ring slot of row t+1 is (t - j0) mod kRIF)
    AdjRow<SPIN, DOT> other;
    int t0 = j0;
    for (; t0 + 2 <= j1; t0 += 2) {
        finish_row(t0, cur, other, bu[0], bn[0]);
        finish_row(t0 + 1, other, cur, bu[1 % kRIF], bn[1 % kRIF]);
    }
    if (t0 < j1) finish_row(t0, cur, other, bu[0], bn[0]);

    // fixed-order reduction over the wavefront, one slot per tile
    if constexpr (SPIN || DOT) {
        for (int off = kWave / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) dlda_slots[(size_t)chunk * A.n_strips + strip] += acc;
    }
}

// Two adjoint steps per pass, cotangents only (temporal blocking, as the
// forward two-step pass): sweep A takes lambda^{m+2} row by row and
// completes lambda^{m+1}, which goes from registers into sweep B, one row
// behind, completing lambda^m.  A covers rows j0-1 .. j1 (reading
// j0-2 .. j1+1), B writes j0 .. j1-1; A's results are valid on lanes 1..62
// and B's on 2..61 (60-column strips).  Every quantity is formed by the same
// expressions as in lw_adjoint_kernel<false>, so the results are identical.
struct AdjCot {
    cd np, nq;          // nu at (i, t), radial boundary columns zeroed
    cd lhq;             // cotangent of the stage-1 Pi value at the half
    cd up, dn;          // stage-2 theta-stencil pieces to rows t+1, t-1
    cd uph, dnh;        // stage-1 theta-stencil pieces to rows t+1, t-1
    Sig si, sh;         // 1/Sigma, 1/Sigma^2 at the integer and half point
    Ang g;              // angular factors of the row (wavefront-uniform)
};

// DOT: also the spin gradient's terms of both steps from stored tangents,
// Re <lambda^{m+2}, T_{m+1}> (tan_a, with the input rows as sweep A
// completes them) and Re <lambda^{m+1}, T_m> (tan_b, with sweep B's rows),
// over the owned points, summed per tile into slots.
template <bool DOT, int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    lw_adjoint2_kernel(const double2* __restrict__ nu_in, double2* __restrict__ lam_out, const double* __restrict__ rad, const double* __restrict__ ang,
                       const ExtPoint* __restrict__ ext, const double* __restrict__ gsample_a,
                       const double* __restrict__ gsample_b, const double2* __restrict__ tan_a,
                       const double2* __restrict__ tan_b, double* __restrict__ dlda_slots, AdjScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const TileOf T = tile_of(xcd_block(blockIdx.x, gridDim.x), wpb, wave, A.n_strips, A.n_chunks);
    const int strip = T.strip, chunk = T.chunk;
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols2 - 2 + lane;
    const unsigned long long interior = ((col >= 1) && (col < nr - 1)) ? ~0ull : 0ull;
    const int ci = min(max(col, 0), nr - 1);

    constexpr int kF = 2 * kNumRad;
    extern __shared__ double rad_s[];  // as in lw_adjoint_kernel<false>
    for (int f = wave; f < T.n_slices * kF; f += wpb) {
        const int g = f % kF, kind = g / kNumRad, field = g % kNumRad;
        const int c = min(max((T.s0 + f / kF) * kStripCols2 - 2 + lane, 0), nr - 1);
        rad_s[f * kWave + lane] = rad[((size_t)field * 2 + kind) * P + (kind == 0 ? c : min(c, nr - 2))];
    }
    __syncthreads();
    if (!T.valid) return;  // wavefront-uniform
    const double* slice = rad_s + T.slice * kF * kWave + lane;
    lds_cptr rvi = (lds_cptr)(slice + 0 * kNumRad * kWave);
    lds_cptr rvh = (lds_cptr)(slice + 1 * kNumRad * kWave);

    const bool own = (lane >= 2) && (lane <= kWave - 3) && (col < nr);
    // Owned rows are stored through row resources (the lane's byte offset,
    // or none) without DOT; with DOT, whose tangent rows need the registers,
    // by plain stores under the lane mask (measured: the row resources spill
    // there).
    const int32_t row_bytes = P * (int32_t)sizeof(double2);
    const uint32_t st_off = own ? (uint32_t)col * sizeof(double2) : kOffNone;
    auto put_row = [&](int t, cd wp, cd wq) {
        if constexpr (DOT) {
            if (own) {
                const size_t o = (size_t)t * P + col;
                st_state<KEEP>(lam_out, o, wp);
                st_state<KEEP>(lam_out, o + A.plane, wq);
            }
        } else {
            const size_t o = (size_t)t * P;
            st_row<KEEP>(row_rsrc(lam_out + o, row_bytes), st_off, wp);
            st_row<KEEP>(row_rsrc(lam_out + o + A.plane, row_bytes), st_off, wq);
        }
    };
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const int aE = min(j1, nth - 1);        // last row sweep A completes
    const int last = min(aE + 1, nth - 1);  // last row of lambda^{m+2} read
    const double sg = (double)A.sigma;
    // both sweeps' output rows, j0-1 .. j1
    const unsigned emask = ext_mask(ext, (gsample_a || gsample_b) ? A.n_ext : 0, j0 - 1, j1, strip * kStripCols2 - 2);

    auto ang_row = [&](int t) -> Ang { return load_ang(ang, nth, min(t, nth - 1)); };
    // arrival of a row (as fresh() of lw_adjoint_kernel<false>)
    // The row's coefficients come with it: sweep B's rows are the rows sweep
    // A has just completed, whose coefficients A's finish() built (same
    // expressions, same values), so B takes them instead of rebuilding them.
    auto fresh_k = [&](cd np, cd nq, const Ang& G, Sig si, Sig sh, const Coef& ki, const Coef& kh) -> AdjCot {
        AdjCot R;
        R.si = si;
        R.sh = sh;
        R.g = G;
        R.np = masked(np, interior);
        R.nq = masked(nq, interior);
        const cd sq = cscale(A.dt, R.nq);
        R.up = cscale(ki.a2s + ki.a1s, sq);
        R.dn = cscale(ki.a2s - ki.a1s, sq);
        const cd lhbq = cadd(cscale(A.dt, R.np), cmul(-ki.ctr, ki.cti, sq));
        const cd ldhq = cscale(A.dt_dr * ki.b, R.nq);
        const cd aq = {fma(0.5, lhbq.re, ldhq.re), fma(0.5, lhbq.im, ldhq.im)};
        const cd bq = {fma(0.5, lhbq.re, -ldhq.re), fma(0.5, lhbq.im, -ldhq.im)};
        R.lhq = cadd(aq, from_right(bq));
        const cd tq = cscale(A.hdt, R.lhq);
        R.uph = cscale(kh.a2s + kh.a1s, tq);
        R.dnh = cscale(kh.a2s - kh.a1s, tq);
        return R;
    };
    auto fresh = [&](int t, cd np, cd nq, const Ang& G) -> AdjCot {
        const int o = t & A.zero;
        const Rad Ri = rad_from_lds(rvi, o), Rh = rad_from_lds(rvh, o);
        const Sig si = kerr_sigma(Ri, G), sh = kerr_sigma(Rh, G);
        return fresh_k(np, nq, G, si, sh, kerr_coef(Ri, G, si), kerr_coef(Rh, G, sh));
    };
    // completion of row t (as in lw_adjoint_kernel<false>): the new
    // cotangent, plus E^T g of the output state's sample; ki, kh receive the
    // row's coefficients
    auto finish = [&](int t, const AdjCot& cur, cd below, cd below_h, cd above, cd above_h, const double* gsample,
                      cd& outp, cd& outq, Coef& ki, Coef& kh) {
        {
            const int o = t & A.zero;
            ki = kerr_coef(rad_from_lds(rvi, o), cur.g, cur.si);
            kh = kerr_coef(rad_from_lds(rvh, o), cur.g, cur.sh);
        }
        const cd mid = cmul(-2.0 * ki.a2s - ki.v0r, ki.v0i, cscale(A.dt, cur.nq));
        const cd cnq = cmul(ki.cre, -ki.cim, cur.nq);
        const cd ldhp = {-A.dt_dr * fma(ki.b, cur.np.re, cnq.re), -A.dt_dr * fma(ki.b, cur.np.im, cnq.im)};
        const cd lhbp = cadd3(mid, below, above);
        const cd ap = {fma(0.5, lhbp.re, ldhp.re), fma(0.5, lhbp.im, ldhp.im)};
        const cd bp = {fma(0.5, lhbp.re, -ldhp.re), fma(0.5, lhbp.im, -ldhp.im)};
        const cd lhp = cadd(ap, from_right(bp));
        const cd midh = cmul(-2.0 * kh.a2s - kh.v0r, kh.v0i, cscale(A.hdt, cur.lhq));
        const cd lubp = cadd(lhp, cadd3(midh, below_h, above_h));
        const cd ctq = cmul(-kh.ctr, kh.cti, cur.lhq);
        const cd lubq = {fma(A.hdt, lhp.re, fma(A.hdt, ctq.re, cur.lhq.re)),
                         fma(A.hdt, lhp.im, fma(A.hdt, ctq.im, cur.lhq.im))};
        const cd cq = cmul(kh.cre, -kh.cim, cur.lhq);
        const cd ldp = {-A.hdt_dr * fma(kh.b, lhp.re, cq.re), -A.hdt_dr * fma(kh.b, lhp.im, cq.im)};
        const cd ldq = cscale(A.hdt_dr * kh.b, cur.lhq);
        const cd cP = {fma(0.5, lubp.re, ldp.re), fma(0.5, lubp.im, ldp.im)};
        const cd cQ = {fma(0.5, lubq.re, ldq.re), fma(0.5, lubq.im, ldq.im)};
        const cd dP = {fma(0.5, lubp.re, -ldp.re), fma(0.5, lubp.im, -ldp.im)};
        const cd dQ = {fma(0.5, lubq.re, -ldq.re), fma(0.5, lubq.im, -ldq.im)};
        outp = cadd3(cur.np, dP, from_left(cP));
        outq = cadd3(cur.nq, dQ, from_left(cQ));
        if (gsample != nullptr && emask != 0) {
            for (int e = 0; e < A.n_ext; ++e) {
                if (!((emask >> e) & 1u)) continue;
                const ExtPoint E = ext[e];
                if (t != E.rowa && t != E.rowb) continue;  // wavefront-uniform
                const double wrow = (t == E.rowa) ? E.wa : E.wb;
                const double w = (col == E.col) ? wrow * (1.0 - E.wr) : (col == E.col + 1) ? wrow * E.wr : 0.0;
                outp.re = fma(w, gsample[2 * e], outp.re);
                outp.im = fma(w, gsample[2 * e + 1], outp.im);
            }
        }
    };
    auto load_row = [&](int t, cd& p, cd& q) {
        const size_t o = (size_t)min(max(t, 0), last) * P + ci;
        p = ld(nu_in, o);
        q = ld(nu_in, o + A.plane);
    };
    // a tangent row (DOT), clamped to the grid
    struct TRow {
        cd p, q;
    };
    auto load_tan = [&](const double2* tan, int t, TRow& r) {
        if constexpr (DOT) {
            const size_t o = (size_t)min(max(t, 0), nth - 1) * P + ci;
            r.p = ld(tan, o);
            r.q = ld(tan, o + A.plane);
        }
    };
    double acc = 0.0;  // spin-gradient partial sum of this lane (DOT)
    // Re <cotangent row, tangent row> of an owned row
    auto dot = [&](const AdjCot& c, const TRow& t) {
        if constexpr (DOT) {
            double v = c.np.re * t.p.re + c.np.im * t.p.im;
            v = fma(c.nq.re, t.q.re, fma(c.nq.im, t.q.im, v));
            if (own) acc += v;
        }
    };

    // ---- prologue: A completes rows j0-1 (if j0 > 0) and j0; B takes them
    // as its halo row and its first row -------------------------------------
    AdjCot a_cur, b_cur;
    cd a_below, a_below_h, b_below, b_below_h;
    {
        cd p, q;
        const int aS = max(j0 - 1, 0);
        if (aS > 0) {
            load_row(aS - 1, p, q);
            const AdjCot h = fresh(aS - 1, p, q, ang_row(aS - 1));
            a_below = h.up;
            a_below_h = h.uph;
        }
        load_row(aS, p, q);
        a_cur = fresh(aS, p, q, ang_row(aS));
        if (aS == 0) {
            a_below = cscale(sg, a_cur.dn);
            a_below_h = cscale(sg, a_cur.dnh);
        }
        for (int r = aS; r <= j0; ++r) {  // one or two rows, wavefront-uniform
            AdjCot a_nxt;
            cd above, above_h;
            if (r + 1 < nth) {
                load_row(r + 1, p, q);
                a_nxt = fresh(r + 1, p, q, ang_row(r + 1));
                above = a_nxt.dn;
                above_h = a_nxt.dnh;
            } else {
                above = cscale(sg, a_cur.up);
                above_h = cscale(sg, a_cur.uph);
                a_nxt = a_cur;
            }
            cd vp, vq;
            Coef ki, kh;
            finish(r, a_cur, a_below, a_below_h, above, above_h, gsample_a, vp, vq, ki, kh);
            if (DOT && r == j0) {  // the one owned row the prologue completes
                TRow tr;
                load_tan(tan_a, r, tr);
                dot(a_cur, tr);
            }
            a_below = a_cur.up;
            a_below_h = a_cur.uph;
            const AdjCot ar = a_cur;
            a_cur = a_nxt;
            if (r < j0) {  // B's halo row j0-1
                const AdjCot h = fresh_k(vp, vq, ar.g, ar.si, ar.sh, ki, kh);
                b_below = h.up;
                b_below_h = h.uph;
            } else {
                b_cur = fresh_k(vp, vq, ar.g, ar.si, ar.sh, ki, kh);
                if (r == 0) {
                    b_below = cscale(sg, b_cur.dn);
                    b_below_h = cscale(sg, b_cur.dnh);
                }
            }
        }
    }

    // ---- main sweep: A completes row r, B row r-1; the row states swap
    // roles from row to row instead of being copied --------------------------
    cd rp[2], rq[2];
    load_row(j0 + 2, rp[0], rq[0]);
    load_row(j0 + 3, rp[1], rq[1]);
    // tangent rows (DOT): step_row(r) finds T_{m+1} row r in ta and T_m row
    // r-1 in tb, and loads the next rows into them once used
    TRow ta, tb;
    load_tan(tan_a, j0 + 1, ta);
    load_tan(tan_b, j0, tb);
    Ang g_next = ang_row(j0 + 2);
    auto step_row = [&](int r, cd& lp, cd& lq, AdjCot& ac, AdjCot& an, AdjCot& bc, AdjCot& bn, TRow& tar,
                        TRow& tbr) {
        cd above, above_h;
        const Ang g1 = g_next;
        g_next = ang_row(r + 2);
        if (r + 1 < nth) {
            an = fresh(r + 1, lp, lq, g1);
            above = an.dn;
            above_h = an.dnh;
        } else {
            above = cscale(sg, ac.up);
            above_h = cscale(sg, ac.uph);
            an = ac;  // unused: the sweep ends with this row
        }
        load_row(r + 3, lp, lq);
        cd vp, vq;
        Coef ki, kh;
        finish(r, ac, a_below, a_below_h, above, above_h, gsample_a, vp, vq, ki, kh);
        if (r < j1) dot(ac, tar);  // wavefront-uniform: row j1 is a halo row of sweep A
        load_tan(tan_a, r + 1, tar);
        a_below = ac.up;
        a_below_h = ac.uph;

        bn = fresh_k(vp, vq, ac.g, ac.si, ac.sh, ki, kh);
        cd wp, wq;
        finish(r - 1, bc, b_below, b_below_h, bn.dn, bn.dnh, gsample_b, wp, wq, ki, kh);
        dot(bc, tbr);
        load_tan(tan_b, r, tbr);
        put_row(r - 1, wp, wq);
        b_below = bc.up;
        b_below_h = bc.uph;
    };
    auto last_row = [&](const AdjCot& bc, const TRow& tbr) {  // the grid's last row: B with the pole ghost row
        cd wp, wq;
        Coef ki, kh;
        finish(nth - 1, bc, b_below, b_below_h, cscale(sg, bc.up), cscale(sg, bc.uph), gsample_b, wp, wq, ki, kh);
        dot(bc, tbr);
        put_row(nth - 1, wp, wq);
    };
    AdjCot a_oth, b_oth;
    int r0 = j0 + 1;
    // Without DOT, enter the row loop as its iterations end: the ring's first
    // row loaded, its second still in flight, so that the compiler's wait at
    // the loop head, which must suit both ways in, does not drain the ring.
    if constexpr (!DOT) __builtin_amdgcn_s_waitcnt(waitcnt_vm(2));
    for (; r0 + 1 <= aE; r0 += 2) {
        step_row(r0, rp[0], rq[0], a_cur, a_oth, b_cur, b_oth, ta, tb);
        step_row(r0 + 1, rp[1], rq[1], a_oth, a_cur, b_oth, b_cur, ta, tb);
    }
    if (r0 <= aE) {
        step_row(r0, rp[0], rq[0], a_cur, a_oth, b_cur, b_oth, ta, tb);
        if (j1 == nth) last_row(b_oth, tb);
    } else if (j1 == nth) {
        last_row(b_cur, tb);
    }

    // fixed-order reduction over the wavefront, one slot per tile
    if constexpr (DOT) {
        for (int off = kWave / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) dlda_slots[(size_t)chunk * A.n_strips + strip] += acc;
    }
}

// One Lax-Wendroff step, u^{m+1} = A u^m, that also writes the derivative of
// the step with respect to the spin at fixed input, T_m = (dA/da) u^m: the
// spin gradient is then dL/da = sum_m Re <lambda^{m+1}, T_m>, a dot product
// the reverse sweep forms from the cotangents it computes anyway.  With
// stage 1 h = ubar - dt/2 [D delta/dr - S(ubar)] at the halves and stage 2
// u' = u - dt [D dh/dr - S(hbar)],
//   dh = -dt/2 [D' delta/dr - S'(ubar)]                       (halves)
//   T  = -dt [D' dh/dr + D d(dh)/dr - S'(hbar) - S(d(h)bar)]   (columns)
// with D', S' the operators of the a-derivatives of the coefficients (the
// Phi row of S' vanishes) and T = 0 on the radial boundary columns.  The
// sweep is that of the one-step forward kernel (64-column strips numbered
// strip-fastest, theta rows in order, the same expressions, so u^{m+1} equals
// its result bit for bit); each lane holds the radial factors of its column
// and half point in registers for the whole tile and their a-derivatives in
// its own part of the wavefront's LDS slice (written and read by the same
// lane: no barrier).

struct TanRow {
    cd p, q;      // u^m at (i, t)
    cd ubp;       // stage-1 average of Phi at the half point i+1/2
    cd hbp, dhp;  // mean and difference of stage-1 Phi at i-1/2, i+1/2
    cd x;         // stage-1 Pi at i+1/2 except its row-(t+1) term: h_Pi = x + wp ubp(t+1)
    double wp;
    cd tbp, tdp;  // the same mean and difference of the a-derivative of stage-1 Phi
    cd tx;        // a-derivative of x
    double twp;   // a-derivative of wp
    Ang g;        // angular factors of row t (wavefront-uniform)
};

template <int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    lw_tangent_kernel(const double2* __restrict__ u_in, double2* __restrict__ u_out, double2* __restrict__ t_out,
                      const double* __restrict__ rad, const double* __restrict__ rad_da,
                      const double* __restrict__ ang, AdjScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x / kWave));
    const int strip = tile % A.n_strips;
    const int chunk = tile / A.n_strips;
    if (chunk >= A.n_chunks) return;  // tiles beyond the last
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols - 1 + lane;
    // Lanes outside the grid read the clamped edge column; their values
    // reach only the radial boundary columns of both outputs, which are zero.
    const int ci = min(max(col, 0), nr - 1);
    const int hi = min(max(col, 0), nr - 2);
    // radial factors of this lane's column and half point; their
    // a-derivatives go to the wavefront's LDS slice [integer/half][field][lane]
    const Rad Vi = load_rad(rad, P, 0, ci), Vh = load_rad(rad, P, 1, hi);
    extern __shared__ double rad_s[];
    double* ds = rad_s + (threadIdx.x / kWave) * 2 * kNumRad * kWave + lane;
#pragma unroll
    for (int f = 0; f < kNumRad; ++f) {
        ds[f * kWave] = rad_da[((size_t)f * 2 + 0) * P + ci];
        ds[(kNumRad + f) * kWave] = rad_da[((size_t)f * 2 + 1) * P + hi];
    }
    lds_cptr rdi = (lds_cptr)ds, rdh = (lds_cptr)(ds + kNumRad * kWave);

    const bool store_ok = (lane >= 1) && (lane <= kWave - 2) && (col < nr);
    const bool boundary = (col == 0) || (col == nr - 1);
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const double sg = (double)A.sigma;
    const int last = (j1 < nth) ? j1 : nth - 1;  // last row this tile reads

    auto ang_row = [&](int t) -> Ang { return load_ang(ang, nth, min(t, nth - 1)); };

    // Arrival of row t: stage-1 pieces (the forward kernel's expressions)
    // and their a-derivatives.  A halo row needs only ubp, hbp and tbp.
    auto fresh = [&](int t, cd p, cd q, cd ubp_prev, const Ang& G) -> TanRow {
        TanRow R;
        R.p = p;
        R.q = q;
        R.g = G;
        const Sig sh = kerr_sigma(Vh, G);
        const Coef kh = kerr_coef(Vh, G, sh);
        const Coef dkh = kerr_coef_da_reg(Vh, rad_from_lds(rdh, t & A.zero), G, sh, kh);
        const cd pr = from_right(p), qr = from_right(q);
        R.ubp = cavg(p, pr);
        const cd ubq = cavg(q, qr);
        const cd dp = csub(pr, p);
        const double tb = A.hdt_dr * kh.b;
        const cd hp = {fma(-tb, dp.re, fma(A.hdt, ubq.re, R.ubp.re)), fma(-tb, dp.im, fma(A.hdt, ubq.im, R.ubp.im))};
        const cd hpl = from_left(hp);
        R.hbp = cavg(hp, hpl);
        R.dhp = csub(hp, hpl);
        // d/da h_Phi = -dt/2 db delta_Phi / dr
        const double ttb = A.hdt_dr * dkh.b;
        const cd thp = {-ttb * dp.re, -ttb * dp.im};
        const cd thpl = from_left(thp);
        R.tbp = cavg(thp, thpl);
        R.tdp = csub(thp, thpl);
        const cd dq = csub(qr, q);
        const cd um = (t == 0) ? cscale(sg, R.ubp) : ubp_prev;
        const cd dq1 = d_pi(kh, dp, dq);
        const cd s1 = s_pi(kh, um, R.ubp, cd{0.0, 0.0}, ubq);
        R.x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, ubq.re)), fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, ubq.im))};
        R.wp = A.hdt * (kh.a2s + kh.a1s);
        // d/da h_Pi = -dt/2 [ (dc delta_Phi - db delta_Pi)/dr - S'(ubar) ]
        const cd tq1 = d_pi(dkh, dp, dq);
        const cd ts1 = s_pi(dkh, um, R.ubp, cd{0.0, 0.0}, ubq);
        R.tx = {fma(A.hdt, ts1.re, -A.hdt_dr * tq1.re), fma(A.hdt, ts1.im, -A.hdt_dr * tq1.im)};
        R.twp = A.hdt * (dkh.a2s + dkh.a1s);
        return R;
    };

    // ---- prologue: rows j0-1 (halo or ghost) and j0 ---------------------
    cd hbp_m, tbp_m;  // hbar_Phi and its a-derivative at row t-1
    TanRow cur;
    {
        cd ubp_prev = {0.0, 0.0};
        if (j0 > 0) {
            const size_t o = (size_t)(j0 - 1) * P + ci;
            const TanRow rm = fresh(j0 - 1, ld(u_in, o), ld(u_in, o + A.plane), ubp_prev, ang_row(j0 - 1));
            ubp_prev = rm.ubp;
            hbp_m = rm.hbp;
            tbp_m = rm.tbp;
        }
        const size_t o = (size_t)j0 * P + ci;
        cur = fresh(j0, ld(u_in, o), ld(u_in, o + A.plane), ubp_prev, ang_row(j0));
        if (j0 == 0) {
            hbp_m = cscale(sg, cur.hbp);
            tbp_m = cscale(sg, cur.tbp);
        }
    }
    Ang g_next = ang_row(j0 + 1);  // angular factors one row ahead
    cd bp[2], bq[2];               // rows j0+1, j0+2 in flight
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const size_t o = (size_t)min(j0 + 1 + k, last) * P + ci;
        bp[k] = ld(u_in, o);
        bq[k] = ld(u_in, o + A.plane);
    }

    // Row t is in cur; row t+1 arrives into nxt (roles alternate from row to
    // row, so no row state is copied); rp, rq: ring slot of row t+1, refilled
    // with row t+3.
    auto finish_row = [&](int t, TanRow& cur, TanRow& nxt, cd& rp, cd& rq) {
        cd ubp_p, hbp_p, tbp_p;
        const Ang g1 = g_next;
        g_next = ang_row(t + 2);
        if (t + 1 < nth) {
            nxt = fresh(t + 1, rp, rq, cur.ubp, g1);
            ubp_p = nxt.ubp;
            hbp_p = nxt.hbp;
            tbp_p = nxt.tbp;
        } else {  // pole ghost row
            ubp_p = cscale(sg, cur.ubp);
            hbp_p = cscale(sg, cur.hbp);
            tbp_p = cscale(sg, cur.tbp);
            nxt = cur;  // unused: the sweep ends with this row
        }
        {
            const size_t o = (size_t)min(t + 3, last) * P + ci;
            rp = ld(u_in, o);
            rq = ld(u_in, o + A.plane);
        }
        const Sig si = kerr_sigma(Vi, cur.g);
        const Coef ki = kerr_coef(Vi, cur.g, si);
        const Coef dki = kerr_coef_da_reg(Vi, rad_from_lds(rdi, t & A.zero), cur.g, si, ki);

        // stage 1, Pi component at the halves, and its a-derivative
        const cd hq = {fma(cur.wp, ubp_p.re, cur.x.re), fma(cur.wp, ubp_p.im, cur.x.im)};
        const cd hql = from_left(hq);
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);
        const cd thq = {fma(cur.twp, ubp_p.re, cur.tx.re), fma(cur.twp, ubp_p.im, cur.tx.im)};
        const cd thql = from_left(thq);
        const cd tbq = cavg(thq, thql);
        const cd tdq = csub(thq, thql);

        // stage 2 (the forward kernel's expressions)
        const double tb = A.dt_dr * ki.b;
        cd np = {fma(-tb, cur.dhp.re, fma(A.dt, hbq.re, cur.p.re)), fma(-tb, cur.dhp.im, fma(A.dt, hbq.im, cur.p.im))};
        const cd dq2 = d_pi(ki, cur.dhp, dhq);
        const cd s2 = s_pi(ki, hbp_m, cur.hbp, hbp_p, hbq);
        cd nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, cur.q.re)), fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, cur.q.im))};
        // T_Phi = -dt/dr (db dh_Phi + b d(dh)_Phi) + dt d(h)bar_Pi
        cd tp = {fma(-A.dt_dr, fma(dki.b, cur.dhp.re, ki.b * cur.tdp.re), A.dt * tbq.re),
                 fma(-A.dt_dr, fma(dki.b, cur.dhp.im, ki.b * cur.tdp.im), A.dt * tbq.im)};
        // T_Pi = -dt/dr [D'(dh) + D(d(dh))]_Pi + dt [S'(hbar) + S(d(h)bar)]
        const cd e1 = d_pi(dki, cur.dhp, dhq), e2 = d_pi(ki, cur.tdp, tdq);
        const cd f1 = s_pi(dki, hbp_m, cur.hbp, hbp_p, hbq), f2 = s_pi(ki, tbp_m, cur.tbp, tbp_p, tbq);
        cd tq = {fma(A.dt, f1.re + f2.re, -A.dt_dr * (e1.re + e2.re)),
                 fma(A.dt, f1.im + f2.im, -A.dt_dr * (e1.im + e2.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
            tp = {0.0, 0.0};
            tq = {0.0, 0.0};
        }
        if (store_ok) {
            const size_t so = (size_t)t * P + col;
            st_state<KEEP>(u_out, so, np);
            st_state<KEEP>(u_out, so + A.plane, nq);
            st(t_out, so, tp);
            st(t_out, so + A.plane, tq);
        }
        hbp_m = cur.hbp;
        tbp_m = cur.tbp;
    };

    TanRow other;
    int t0 = j0;
    for (; t0 + 2 <= j1; t0 += 2) {
        finish_row(t0, cur, other, bp[0], bq[0]);
        finish_row(t0 + 1, other, cur, bp[1], bq[1]);
    }
    if (t0 < j1) finish_row(t0, cur, other, bp[0], bq[0]);
}


// lam_Phi += E^T g for every extraction point, in point order (one thread).
__global__ void extract_adjoint_kernel(double2* __restrict__ lam, int pitch, const ExtPoint* __restrict__ pts, int n,
                                       const double2* __restrict__ g) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int e = 0; e < n; ++e) {
        const ExtPoint E = pts[e];
        const double2 gv = g[e];
        for (int r = 0; r < 2; ++r) {
            const int row = r == 0 ? E.rowa : E.rowb;
            if (row < 0) continue;
            const double w = r == 0 ? E.wa : E.wb;
            double2* a = &lam[(size_t)row * pitch + E.col];
            double2* b = &lam[(size_t)row * pitch + E.col + 1];
            const double wa = w * (1.0 - E.wr), wb = w * E.wr;
            a->x = fma(wa, gv.x, a->x);
            a->y = fma(wa, gv.y, a->y);
            b->x = fma(wb, gv.x, b->x);
            b->y = fma(wb, gv.y, b->y);
        }
    }
}

// Sum of the spin-gradient slots in a fixed order (one workgroup), added to *out.
__global__ void reduce_slots_kernel(const double* __restrict__ slots, int n, double* __restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += slots[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += part[0];
}

// Zero the radial boundary columns of a state.
__global__ void zero_radial_boundary_kernel(double2* __restrict__ u, int nr, int nth, int pitch) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nth) return;
    const double2 z = {0.0, 0.0};
    const size_t plane = (size_t)nth * pitch;
    const size_t a = (size_t)j * pitch, b = (size_t)j * pitch + nr - 1;
    u[a] = z;
    u[a + plane] = z;
    u[b] = z;
    u[b + plane] = z;
}

}  // namespace


hipError_t launch_adjoint(const AdjArgs& a, int waves_per_block, AdjMode mode, hipStream_t s) {
    dim3 grid, block;
    size_t lds;
    const bool spin = mode == AdjMode::kSpin;
    adjoint_launch_shape(a.k, waves_per_block, (spin ? 4 : 2) * kNumRad, &grid, &block, &lds);
    const bool keep = a.k.keep != 0;
    auto pick = [&](auto k0, auto k1) { return keep ? k1 : k0; };
    auto kern = spin ? pick(lw_adjoint_kernel<true, false, 0>, lw_adjoint_kernel<true, false, 1>)
                     : (mode == AdjMode::kTangentDot ? pick(lw_adjoint_kernel<false, true, 0>,
                                                            lw_adjoint_kernel<false, true, 1>)
                                                     : pick(lw_adjoint_kernel<false, false, 0>,
                                                            lw_adjoint_kernel<false, false, 1>));
    hipLaunchKernelGGL(kern, grid, block, lds, s, a.nu_in, a.u_in, a.lam_out, a.rad, a.rad_da, a.ang, a.slots, a.ext,
                       a.gsample, a.k);
    return hipGetLastError();
}

hipError_t launch_adjoint2(const AdjArgs& a, const double* gsample_b, const double2* tan_b, int waves_per_block,
                           hipStream_t s) {
    dim3 grid, block;
    size_t lds;
    adjoint_launch_shape(a.k, waves_per_block, 2 * kNumRad, &grid, &block, &lds);
    const bool keep = a.k.keep != 0;
    auto kern = a.u_in ? (keep ? lw_adjoint2_kernel<true, 1> : lw_adjoint2_kernel<true, 0>)
                       : (keep ? lw_adjoint2_kernel<false, 1> : lw_adjoint2_kernel<false, 0>);
    hipLaunchKernelGGL(kern, grid, block, lds, s, a.nu_in, a.lam_out, a.rad, a.ang, a.ext, a.gsample, gsample_b,
                       a.u_in, tan_b, a.slots, a.k);
    return hipGetLastError();
}

hipError_t launch_tangent(const double2* u_in, double2* u_out, double2* t_out, const AdjArgs& a, int waves_per_block,
                          hipStream_t s) {
    const int64_t tiles = (int64_t)a.k.n_strips * a.k.n_chunks;
    const dim3 block(kWave * waves_per_block), grid((unsigned)((tiles + waves_per_block - 1) / waves_per_block));
    const size_t lds = (size_t)waves_per_block * 2 * kNumRad * kWave * sizeof(double);
    hipLaunchKernelGGL(a.k.keep ? lw_tangent_kernel<1> : lw_tangent_kernel<0>, grid, block, lds, s, u_in, u_out, t_out,
                       a.rad, a.rad_da, a.ang, a.k);
    return hipGetLastError();
}


hipError_t launch_extract_adjoint(double2* lam, int pitch, const ExtPoint* pts, int n, const double2* g,
                                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(extract_adjoint_kernel, dim3(1), dim3(64), 0, s, lam, pitch, pts, n, g);
    return hipGetLastError();
}

hipError_t launch_reduce_slots(const double* slots, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_slots_kernel, dim3(1), dim3(256), 0, s, slots, n, out);
    return hipGetLastError();
}

hipError_t launch_zero_radial_boundary(double2* u, int nr, int nth, int pitch, hipStream_t s) {
    hipLaunchKernelGGL(zero_radial_boundary_kernel, dim3((nth + 255) / 256), dim3(256), 0, s, u, nr, nth, pitch);
    return hipGetLastError();
}

}  // namespace teuk
