// The statistic of an explicit template list: the uniform random template
// bank of Sec. 2, where every template has its own (f0, tau, n, sky) and no
// per-group table can be shared.
#include "ltgw_gather.h"
#include "ltgw_list.h"
#include "ddpow.h"

#pragma clang fp contract(off)

namespace ltgw {

// Lane q evaluates template perm[q] over every selected detector and segment
// with the lattice's arithmetic, in its order:
//   t < T0: masked (g = 0, so the column falls out of band)
//   u = 1 + (t - T0)/tau, e = 1/(1 - n), g = RN(u^e)            (Eq. 1)
//   D = 1 + ((vx nx + vy ny) + vz nz)/c, H = RN(RN(g D) T_sft)   (Eq. 2)
//   x = f0 H, column = trunc(x + 1.5 - k_lo), gather, FP32 sums over chunks
//   of 32 segments carried in FP64                               (Sec. 2)
// so a template of a lattice gets that lattice's s, c and N bit for bit (the
// two quotients come from reciprocals by div_rn, which equals the division).
// The power is correctly rounded per segment (the fast phase, and the
// double-double phase where that cannot decide; both counted), which makes
// this mode bound by FP64 arithmetic.  Sorting the list by f0 (the caller's
// perm) keeps neighbouring lanes on neighbouring columns for the gathers.
// ANT: some detector carries antenna-pattern weights.  Without, the kernel
// holds none of their per-detector values, which leaves the scalar registers
// to the power's constants (else they spill into vector-register lanes).
// DOP: every detector has a Doppler table (one sky direction for the whole
// list), read per segment instead of formed per template.
template <int STORE, bool ANT, bool DOP>
__global__ __launch_bounds__(256) void template_list_kernel(const ListArgs a) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = q < a.n;
    const int32_t o = live ? a.perm[q] : a.perm[0];
    const ltgw_template T = a.tpl[o];
    const double e = 1.0 / (1.0 - T.brake);
    const double rtau = 1.0 / T.tau;  // RN(1/tau): the per-segment quotients by div_rn
    double s = 0.0, w1 = 0.0, w2 = 0.0;
    int cnt = 0, nin = 0;
    for (int d = 0; d < a.n_det; ++d) {
        const ListDet D = a.det[d];
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)D.store, Store<STORE>::kBytes, D.n_bins + 2, kBufDword3);
        const unsigned nb = (unsigned)D.n_bins;
        for (int j0 = 0; j0 < D.n_seg; j0 += kChunk) {
            const int je = min(j0 + kChunk, D.n_seg);
            float sc = 0.0f, w1c = 0.0f, w2c = 0.0f;
            for (int j = j0; j < je; ++j) {
                const double t = uniform_load(D.t, j);
                double g = 0.0;
                if (!(t < a.t0)) {
                    const double dt = t - a.t0;
                    const double qq = div_rn(dt, T.tau, rtau);
                    const double u = 1.0 + qq;
                    int und = 0;
                    int slow = 0;
                    g = pow_cr(u, e, &und, &slow);
                    if (und) atomicAdd(a.pow_counts, 1ull);
                    if (slow) atomicAdd(a.pow_counts + 1, 1ull);
                }
                double Df;
                if (DOP) {
                    Df = uniform_load(D.dop, j);
                } else {
                    const double va = uniform_load(D.v, 3 * j + 0) * T.sky[0];
                    const double vb = uniform_load(D.v, 3 * j + 1) * T.sky[1];
                    const double vz = uniform_load(D.v, 3 * j + 2) * T.sky[2];
                    const double vn = (va + vb) + vz;
                    const double r = div_rn(vn, kC, kInvC);
                    Df = 1.0 + r;
                }
                const double h = g * Df;
                const double H = h * D.t_sft;
                const double x = T.f0 * H;
                const double vv = x + D.cshift;
                const unsigned idx = (unsigned)__double2int_rz(vv);
                const float p = Store<STORE>::get(rs, (int)idx, j * D.pitch_bytes, cnt);
                float wq = uniform_load(D.wq, j), wv = uniform_load(D.w, j);
                if (ANT && D.era)  // antenna-pattern weights for this template's sky direction
                    antenna_weights(D.arms, uniform_load(D.era, j), T.sky[0], T.sky[1], T.sky[2], wv,
                                    uniform_load(D.scale, j), wv, wq);
                sc = __builtin_fmaf(wq, p, sc);
                const bool inb = (idx - 1u) < nb;
                nin += inb ? 1 : 0;
                const float wj = inb ? wv : 0.0f;
                w1c += wj;
                w2c = __builtin_fmaf(wj, wj, w2c);
            }
            s += (double)sc;
            w1 += (double)w1c;
            w2 += (double)w2c;
        }
    }
    // the in-band total of the list (diagnostics): one atomic per wavefront
    unsigned long long mine = live ? (unsigned long long)nin : 0ull;
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(a.in_band_total, mine);
    if (!live) return;
    a.s[o] = s;
    a.c[o] = cnt;
    a.n_in[o] = nin;
    a.w1[o] = w1;
    a.w2[o] = w2;
    if (a.out_s) a.out_s[o] = (float)s;
    if (a.out_c) a.out_c[o] = cnt;
    if (a.out_n) a.out_n[o] = nin;
}

template <int STORE>
static void launch_list_store(bool ant, bool dop, const ListArgs &a, dim3 grid, hipStream_t st) {
    if (ant)
        hipLaunchKernelGGL((template_list_kernel<STORE, true, false>), grid, dim3(256), 0, st, a);
    else if (dop)
        hipLaunchKernelGGL((template_list_kernel<STORE, false, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((template_list_kernel<STORE, false, false>), grid, dim3(256), 0, st, a);
}

hipError_t launch_template_list(int store, const ListArgs &a, hipStream_t st) {
    if (a.n < 1 || a.n > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.n + 255) / 256));
    bool ant = false, dop = true;
    for (int d = 0; d < a.n_det; ++d) {
        ant = ant || a.det[d].era != nullptr;
        dop = dop && a.det[d].dop != nullptr;
    }
    if (store == LTGW_STORE_F32)
        launch_list_store<LTGW_STORE_F32>(ant, dop, a, grid, st);
    else if (store == LTGW_STORE_BF16)
        launch_list_store<LTGW_STORE_BF16>(ant, dop, a, grid, st);
    else
        launch_list_store<LTGW_STORE_FP8>(ant, dop, a, grid, st);
    return hipGetLastError();
}

}  // namespace ltgw
