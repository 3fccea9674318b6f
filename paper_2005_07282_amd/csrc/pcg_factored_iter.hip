// Jacobi-PCG with the Jacobi step replaced by a factored preconditioner
// M^-1 = G G^T + eps I (the learned preconditioner's form; G^T is given
// explicitly): the iteration's kernels after the SpMV+<d,w> kernel. S5 becomes
// t = G^T r, s = G t, z_i = fma(eps, r_i, s_i), each product a row-wise fma
// chain in storage order from +0 (Section 4.3), so the iteration stays
// reproducible given G. The SpMV and direction kernels are the Jacobi solver's.
#include "pcg_factored.hpp"

namespace rpcg {

// t = G^T r (one row per thread).
__global__ void k_fac_gt(int n, FacPre Pr, const double *__restrict__ r, double *__restrict__ t, const PcgState *st)
{
    if (st->done) return;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        t[i] = csr_row(Pr.gt_rp, Pr.gt_col, Pr.gt_val, r, i);
}

// Iteration l after the SpMV kernel, first launch. Prologue: merge delta,
// rho = beta / delta. Per row i: S3 x_i = fma(rho, d_i, x_i); S4 r_i =
// fma(-rho, w_i, r_i) into the other r buffer, with the partials of
// tau = <r, r> (wt); and t_i = (G^T r)_i, the fma chain of row i of G^T in
// storage order from +0 over the new r. r_old is only read, so a row
// recomputes each neighbour's new r_j from w_j and r_old_j (the same bits as
// the stored one) instead of waiting for a grid-wide barrier.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_fac_update(int l, int n, FacPre Pr, PcgVecs<double> v, const double *__restrict__ r_old, double *__restrict__ r_new,
             double *__restrict__ t, PcgState *st, SlotView sd, int Gd, SlotView wt, bool ee, bool capture)
{
    __shared__ RedShared sh;
    if (wg_read_flag(&st->done, sh)) return;
    long long esc_d = 0;
    const double delta = merge_slots<MODE, P>(sd, Gd, ee, capture, sh.acc[0], &esc_d, &st->flags, sh, 0);
    const bool bad = (st->flags & FLAG_NONFINITE) || !is_finite_bits(delta);
    const bool breakdown = !(delta > 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->escapes += esc_d;
        if (capture && esc_d > 0) st->fallbacks += 1;
        st->delta = delta;
        if (bad) { st->status = -6; st->done = 1; }
        else if (breakdown) { st->status = -5; st->done = 1; }
    }
    if (bad || breakdown) return;
    const double rho = v.beta_hist[l] / delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho = rho;
    zero_acc(sh.acc[1]);
    __syncthreads();
    LaneDot<MODE, P> Lt;
    Lt.init();
    const double *__restrict__ w = v.w;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        v.x[i] = __builtin_fma(rho, v.d[i], v.x[i]);              // S3
        const double ri = __builtin_fma(-rho, w[i], r_old[i]);     // S4
        r_new[i] = ri;
        Lt.add(ri, ri, sh.acc[1], ee, capture);                    // S8
        double ti = 0.0;                                           // (G^T r)_i
        const int m1 = Pr.gt_rp[i + 1];
        for (int m = Pr.gt_rp[i]; m < m1; ++m) {
            const int j = Pr.gt_col[m];
            ti = __builtin_fma(Pr.gt_val[m], __builtin_fma(-rho, w[j], r_old[j]), ti);
        }
        t[i] = ti;
    }
    block_finish<MODE, P>(Lt, sh.acc[1], wt, blockIdx.x, ee, capture, &st->flags, sh);
}

hipError_t launch_fac_update(int mode, int l, int n, const FacPre &Pr, const PcgVecs<double> &v, double *r_new,
                             double *t, PcgState *st, const DotWs &wsd, int Gd, const DotWs *ws, int stride,
                             const LaunchCfg &c)
{
    SlotView sd{wsd, stride}, s0{ws[0], stride}, s1{ws[1], stride};
    PcgVecs<double> vz = v;
    vz.r = r_new;
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        k_fac_update<M, PP><<<c.grid, c.block, 0, c.stream>>>(l, n, Pr, v, v.r, r_new, t, st, sd, Gd, s1,
                                                              c.early_exit, c.fallback);
        k_fac_z<M, PP, false><<<c.grid, c.block, 0, c.stream>>>(n, Pr, vz, t, st, s0, c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
