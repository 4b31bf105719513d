// gfx950 forward-mode derivative of the Lax-Wendroff step (arXiv:1010.3816,
// Eqs. (lw1)-(lw2) with the boundary conditions) with respect to the spin a:
// the state and its a-derivative advance together, one pass per step.
// Compiled on its own with the machine scheduler's occupancy-first strategy:
// the two states' row data fit the registers of two wavefronts per SIMD only
// when scheduled for occupancy (the default schedule spills).
#include "adjoint_common.hpp"

namespace teuk {
namespace {

// Forward-mode derivative with respect to the spin: one step of the state,
// u^{m+1} = A u^m, and of its a-derivative v = du/da,
//   v^{m+1} = A v^m + (dA/da) u^m.
// Stage 2 is linear in the stage-1 values, so with W = S1(v) + (dS1/da) u
// (the a-derivative of the stage-1 result along the trajectory)
//   v^{m+1} = v^m - dt [D' dh/dr + D dW/dr - S'(hbar) - S(Wbar)],
// the tangent step's T with W in place of d(h) and v^m added.  The sweep,
// tiles and u^{m+1} are those of lw_tangent_kernel (bit for bit); the
// samples of u^m and v^m at the tile's (at most one) extraction point are
// fused as in the forward kernels.
#ifndef TEUK_SPIN_TANGENT_RING
#define TEUK_SPIN_TANGENT_RING 1
#endif
constexpr int kFtRing = TEUK_SPIN_TANGENT_RING;  // rows of u and v loaded ahead (1 or 2)
static_assert(kFtRing == 1 || kFtRing == 2, "one or two rows in flight");
struct FtRow {
    cd p, q;      // u^m at (i, t)
    cd vp, vq;    // v^m at (i, t)
    cd ubp, ubv;  // stage-1 averages of Phi (u, v) at the half point i+1/2
    cd hbp, dhp;  // mean and difference of stage-1 Phi of u at i-1/2, i+1/2
    cd x;         // stage-1 Pi of u at i+1/2 except its row-(t+1) term: h_Pi = x + wp ubp(t+1)
    double wp;
    cd wbp, wdp;  // mean and difference of W_Phi
    cd wx;        // W_Pi except its row-(t+1) terms: W_Pi = wx + wp ubv(t+1) + twp ubp(t+1)
    double twp;   // a-derivative of wp
    Ang g;        // angular factors of row t (wavefront-uniform)
};

template <int KEEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    lw_spin_tangent_kernel(const double2* __restrict__ u_in, const double2* __restrict__ v_in,
                           double2* __restrict__ u_out, double2* __restrict__ v_out,
                           const double* __restrict__ rad, const double* __restrict__ rad_da,
                           const double* __restrict__ ang, const ExtPoint* __restrict__ ext,
                           double2* __restrict__ series_u, double2* __restrict__ series_v, AdjScalars A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const TileOf T = tile_of(xcd_block(blockIdx.x, gridDim.x), wpb, wave, A.n_strips, A.n_chunks);
    const int strip = T.strip, chunk = T.chunk;
    const int nr = A.nr, nth = A.nth, P = A.pitch;
    const int col = strip * kStripCols - 1 + lane;
    const int ci = min(max(col, 0), nr - 1);
    // the radial tables and their a-derivatives for the workgroup's strips,
    // [strip][value/derivative][integer/half][field][lane], read row by row
    // (the registers go to the second state)
    constexpr int kF = 4 * kNumRad;
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

    const bool store_ok = (lane >= 1) && (lane <= kWave - 2) && (col < nr);
    const bool boundary = (col == 0) || (col == nr - 1);
    // rows through row resources (lane byte offsets: the clamped column for
    // loads; the owned column, or none, for stores)
    const int32_t row_bytes = P * (int32_t)sizeof(double2);
    const uint32_t st_off = store_ok ? (uint32_t)col * sizeof(double2) : kOffNone;
    auto load_row = [&](int t, cd& p, cd& q, cd& vp, cd& vq) {
        const size_t o = (size_t)t * P + ci;
        p = ld(u_in, o);
        q = ld(u_in, o + A.plane);
        vp = ld(v_in, o);
        vq = ld(v_in, o + A.plane);
    };
    const int j0 = chunk * A.rows;
    const int j1 = min(j0 + A.rows, nth);
    const double sg = (double)A.sigma;
    const int last = (j1 < nth) ? j1 : nth - 1;

    // the (at most one) extraction point of this tile, in scalar registers
    int e_id = -1, e_lane = 0, e_ra = -1, e_rb = -1;
    double e_wr = 0.0, e_wa = 0.0, e_wb = 0.0;
    for (int e = 0; e < A.n_ext; ++e) {
        const ExtPoint E = ext[e];
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
    cd acc_u = {0.0, 0.0}, acc_v = {0.0, 0.0};

    auto ang_row = [&](int t) -> Ang { return load_ang(ang, nth, min(t, nth - 1)); };

    // Arrival of row t: stage-1 pieces of u (the forward kernel's
    // expressions), of v, and the a-derivatives of u's; samples of u and v.
    auto fresh = [&](int t, cd p, cd q, cd vp, cd vq, cd ubp_prev, cd ubv_prev, const Ang& G) -> FtRow {
        FtRow R;
        R.p = p;
        R.q = q;
        R.vp = vp;
        R.vq = vq;
        R.g = G;
        const Rad Vh = rad_from_lds(rvh, t & A.zero);
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
        const cd dq = csub(qr, q);
        const cd um = (t == 0) ? cscale(sg, R.ubp) : ubp_prev;
        const cd dq1 = d_pi(kh, dp, dq);
        const cd s1 = s_pi(kh, um, R.ubp, cd{0.0, 0.0}, ubq);
        R.x = {fma(A.hdt, s1.re, fma(-A.hdt_dr, dq1.re, ubq.re)), fma(A.hdt, s1.im, fma(-A.hdt_dr, dq1.im, ubq.im))};
        R.wp = A.hdt * (kh.a2s + kh.a1s);
        // v: the same stage-1 expressions
        const cd vpr = from_right(vp), vqr = from_right(vq);
        R.ubv = cavg(vp, vpr);
        const cd ubvq = cavg(vq, vqr);
        const cd dv = csub(vpr, vp);
        const cd dvq = csub(vqr, vq);
        const cd umv = (t == 0) ? cscale(sg, R.ubv) : ubv_prev;
        // W_Phi = h_Phi(v) - dt/2 db delta_Phi(u) / dr
        const double ttb = A.hdt_dr * dkh.b;
        const cd whp = {fma(-ttb, dp.re, fma(-tb, dv.re, fma(A.hdt, ubvq.re, R.ubv.re))),
                        fma(-ttb, dp.im, fma(-tb, dv.im, fma(A.hdt, ubvq.im, R.ubv.im)))};
        const cd whpl = from_left(whp);
        R.wbp = cavg(whp, whpl);
        R.wdp = csub(whp, whpl);
        // W_Pi without its row-(t+1) terms: x(v) + d/da x(u)
        const cd dq1v = d_pi(kh, dv, dvq);
        const cd s1v = s_pi(kh, umv, R.ubv, cd{0.0, 0.0}, ubvq);
        const cd tq1 = d_pi(dkh, dp, dq);
        const cd ts1 = s_pi(dkh, um, R.ubp, cd{0.0, 0.0}, ubq);
        R.wx = {fma(A.hdt, s1v.re + ts1.re, fma(-A.hdt_dr, dq1v.re + tq1.re, ubvq.re)),
                fma(A.hdt, s1v.im + ts1.im, fma(-A.hdt_dr, dq1v.im + tq1.im, ubvq.im))};
        R.twp = A.hdt * (dkh.a2s + dkh.a1s);
        if (t == e_ra || t == e_rb) {  // wavefront-uniform
            const double w = (t == e_ra) ? e_wa : e_wb;
            acc_u.re = fma(w, fma(e_wr, pr.re - p.re, p.re), acc_u.re);
            acc_u.im = fma(w, fma(e_wr, pr.im - p.im, p.im), acc_u.im);
            acc_v.re = fma(w, fma(e_wr, vpr.re - vp.re, vp.re), acc_v.re);
            acc_v.im = fma(w, fma(e_wr, vpr.im - vp.im, vp.im), acc_v.im);
        }
        return R;
    };

    // ---- prologue: rows j0-1 (halo or ghost) and j0 ---------------------
    cd hbp_m, wbp_m;  // hbar_Phi and Wbar_Phi at row t-1
    FtRow cur;
    {
        cd ubp_prev = {0.0, 0.0}, ubv_prev = {0.0, 0.0};
        if (j0 > 0) {
            cd p, q, vp, vq;
            load_row(j0 - 1, p, q, vp, vq);
            const FtRow rm = fresh(j0 - 1, p, q, vp, vq, ubp_prev, ubv_prev, ang_row(j0 - 1));
            ubp_prev = rm.ubp;
            ubv_prev = rm.ubv;
            hbp_m = rm.hbp;
            wbp_m = rm.wbp;
        }
        cd p, q, vp, vq;
        load_row(j0, p, q, vp, vq);
        cur = fresh(j0, p, q, vp, vq, ubp_prev, ubv_prev, ang_row(j0));
        if (j0 == 0) {
            hbp_m = cscale(sg, cur.hbp);
            wbp_m = cscale(sg, cur.wbp);
        }
    }
    Ang g_next = ang_row(j0 + 1);
    cd bp[2], bq[2], bvp[2], bvq[2];  // rows j0+1 .. j0+kFtRing of u and v in flight
#pragma unroll
    for (int k = 0; k < kFtRing; ++k) load_row(min(j0 + 1 + k, last), bp[k], bq[k], bvp[k], bvq[k]);

    auto finish_row = [&](int t, FtRow& cur, FtRow& nxt, cd& rp, cd& rq, cd& rvp, cd& rvq) {
        cd ubp_p, ubv_p, hbp_p, wbp_p;
        const Ang g1 = g_next;
        g_next = ang_row(t + 2);
        if (t + 1 < nth) {
            nxt = fresh(t + 1, rp, rq, rvp, rvq, cur.ubp, cur.ubv, g1);
            ubp_p = nxt.ubp;
            ubv_p = nxt.ubv;
            hbp_p = nxt.hbp;
            wbp_p = nxt.wbp;
        } else {  // pole ghost row
            ubp_p = cscale(sg, cur.ubp);
            ubv_p = cscale(sg, cur.ubv);
            hbp_p = cscale(sg, cur.hbp);
            wbp_p = cscale(sg, cur.wbp);
            nxt = cur;  // unused: the sweep ends with this row
        }
        load_row(min(t + 1 + kFtRing, last), rp, rq, rvp, rvq);
        const Rad Vi = rad_from_lds(rvi, t & A.zero);
        const Sig si = kerr_sigma(Vi, cur.g);
        const Coef ki = kerr_coef(Vi, cur.g, si);
        const Coef dki = kerr_coef_da_reg(Vi, rad_from_lds(rdi, t & A.zero), cur.g, si, ki);

        // stage 1, Pi component at the halves, of u and of W
        const cd hq = {fma(cur.wp, ubp_p.re, cur.x.re), fma(cur.wp, ubp_p.im, cur.x.im)};
        const cd hql = from_left(hq);
        const cd hbq = cavg(hq, hql);
        const cd dhq = csub(hq, hql);
        const cd whq = {fma(cur.twp, ubp_p.re, fma(cur.wp, ubv_p.re, cur.wx.re)),
                        fma(cur.twp, ubp_p.im, fma(cur.wp, ubv_p.im, cur.wx.im))};
        const cd whql = from_left(whq);
        const cd wbq = cavg(whq, whql);
        const cd wdq = csub(whq, whql);

        // stage 2 of u (the forward kernel's expressions)
        const double tb = A.dt_dr * ki.b;
        cd np = {fma(-tb, cur.dhp.re, fma(A.dt, hbq.re, cur.p.re)), fma(-tb, cur.dhp.im, fma(A.dt, hbq.im, cur.p.im))};
        const cd dq2 = d_pi(ki, cur.dhp, dhq);
        const cd s2 = s_pi(ki, hbp_m, cur.hbp, hbp_p, hbq);
        cd nq = {fma(A.dt, s2.re, fma(-A.dt_dr, dq2.re, cur.q.re)), fma(A.dt, s2.im, fma(-A.dt_dr, dq2.im, cur.q.im))};
        // v' = v - dt/dr (db dh_Phi + b dW_Phi) + dt Wbar_Pi, and the Pi row
        cd nvp = {cur.vp.re + fma(-A.dt_dr, fma(dki.b, cur.dhp.re, ki.b * cur.wdp.re), A.dt * wbq.re),
                  cur.vp.im + fma(-A.dt_dr, fma(dki.b, cur.dhp.im, ki.b * cur.wdp.im), A.dt * wbq.im)};
        const cd e1 = d_pi(dki, cur.dhp, dhq), e2 = d_pi(ki, cur.wdp, wdq);
        const cd f1 = s_pi(dki, hbp_m, cur.hbp, hbp_p, hbq), f2 = s_pi(ki, wbp_m, cur.wbp, wbp_p, wbq);
        cd nvq = {cur.vq.re + fma(A.dt, f1.re + f2.re, -A.dt_dr * (e1.re + e2.re)),
                  cur.vq.im + fma(A.dt, f1.im + f2.im, -A.dt_dr * (e1.im + e2.im))};
        if (boundary) {
            np = {0.0, 0.0};
            nq = {0.0, 0.0};
            nvp = {0.0, 0.0};
            nvq = {0.0, 0.0};
        }
        {
            const size_t o = (size_t)t * P;
            st_row<KEEP>(row_rsrc(u_out + o, row_bytes), st_off, np);
            st_row<KEEP>(row_rsrc(u_out + o + A.plane, row_bytes), st_off, nq);
            st_row<KEEP>(row_rsrc(v_out + o, row_bytes), st_off, nvp);
            st_row<KEEP>(row_rsrc(v_out + o + A.plane, row_bytes), st_off, nvq);
        }
        hbp_m = cur.hbp;
        wbp_m = cur.wbp;
    };

    FtRow other;
    int t0 = j0;
    constexpr int s1 = kFtRing - 1;  // ring slot of the pair's second row
    // Enter the row loop with the ring loaded, as each iteration leaves it
    // apart from its last stores: the compiler's wait at the loop head, which
    // must suit both ways in, then leaves those stores in flight.
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    for (; t0 + 2 <= j1; t0 += 2) {
        finish_row(t0, cur, other, bp[0], bq[0], bvp[0], bvq[0]);
        finish_row(t0 + 1, other, cur, bp[s1], bq[s1], bvp[s1], bvq[s1]);
    }
    if (t0 < j1) finish_row(t0, cur, other, bp[0], bq[0], bvp[0], bvq[0]);

    if (e_id >= 0 && lane == e_lane) {
        if (series_u != nullptr) series_u[e_id] = double2{acc_u.re, acc_u.im};
        if (series_v != nullptr) series_v[e_id] = double2{acc_v.re, acc_v.im};
    }
}

// *out += sum_i Re(conj(g_i) t_i) over count complex values (one workgroup:
// a fixed summation order, so the result does not depend on the launch).
__global__ void __launch_bounds__(256) series_dot_kernel(const double2* __restrict__ g, const double2* __restrict__ t,
                                                         int64_t count, double* __restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s = fma(g[i].x, t[i].x, fma(g[i].y, t[i].y, s));
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += part[0];
}

}  // namespace

hipError_t launch_series_dot(const double2* g, const double2* t, int64_t count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(series_dot_kernel, dim3(1), dim3(256), 0, s, g, t, count, out);
    return hipGetLastError();
}

hipError_t launch_spin_tangent(const double2* u_in, const double2* v_in, double2* u_out, double2* v_out,
                               double2* series_u, double2* series_v, const AdjArgs& a, int waves_per_block,
                               hipStream_t s) {
    dim3 grid, block;
    size_t lds;
    adjoint_launch_shape(a.k, waves_per_block, 4 * kNumRad, &grid, &block, &lds);
    hipLaunchKernelGGL(a.k.keep ? lw_spin_tangent_kernel<1> : lw_spin_tangent_kernel<0>, grid, block, lds, s, u_in,
                       v_in, u_out, v_out, a.rad, a.rad_da, a.ang, a.ext, series_u, series_v, a.k);
    return hipGetLastError();
}

}  // namespace teuk
