// The statistic of an explicit template list: the uniform random template
// bank of Sec. 2, where every template has its own (f0, tau, n, sky) and no
// per-group table can be shared.
#include "ltgw_gather.h"
#include "ltgw_list.h"
#include "ddpow.h"
#include "pow_enclose.h"

#pragma clang fp contract(off)

namespace ltgw {

// segments whose columns and gathers are formed together (divides kChunk)
constexpr int kListBatch = 8;
static_assert(kChunk % kListBatch == 0, "a batch must not straddle a chunk");

// D_j = 1 + v_j.n/c (Eq. 2): the detector's table for a one-sky list, else
// formed from the template's sky direction
template <bool DOP>
__device__ inline double doppler(const ListDet &D, int j, const ltgw_template &T) {
    if (DOP) return uniform_load(D.dop, j);
    const double va = uniform_load(D.v, 3 * j + 0) * T.sky[0];
    const double vb = uniform_load(D.v, 3 * j + 1) * T.sky[1];
    const double vz = uniform_load(D.v, 3 * j + 2) * T.sky[2];
    const double vn = (va + vb) + vz;
    return 1.0 + div_rn(vn, kC, kInvC);
}

// The enclosure's tables as copies in LDS (filled once per workgroup): a
// wavefront's 64 lanes read scattered entries, which LDS serves in a few
// cycles where the constant arrays cost a round trip through the cache.
struct LdsTables {
    const double2 *lg;  // [128] (r_i, RN(-log r_i))
    const double *ex;   // [256] RN(2^(j/256))
    __device__ void log_entry(int i, double *r, double *t) const {
        const double2 v = lg[i];
        *r = v.x;
        *t = v.y;
    }
    __device__ double exp2_entry(int j) const { return ex[j]; }
};

// the column of the track for spin-down factor g; monotone in g
__device__ inline unsigned column(const ListDet &D, const ltgw_template &T, double Df, double g) {
    const double h = g * Df;
    const double H = h * D.t_sft;
    const double x = T.f0 * H;
    return (unsigned)__double2int_rz(x + D.cshift);
}

// Lane q evaluates template perm[q] over every selected detector and segment
// with the lattice's arithmetic, in its order:
//   t < T0: masked (g = 0, so the column falls out of band)
//   u = 1 + (t - T0)/tau, e = 1/(1 - n), g = RN(u^e)            (Eq. 1)
//   D = 1 + ((vx nx + vy ny) + vz nz)/c, H = RN(RN(g D) T_sft)   (Eq. 2)
//   x = f0 H, column = trunc(x + 1.5 - k_lo), gather, FP32 sums over chunks
//   of 32 segments carried in FP64                               (Sec. 2)
// so a template of a lattice gets that lattice's s, c and N bit for bit (the
// two quotients come from reciprocals by div_rn, which equals the division).
// The column is monotone in g, so it is taken at both ends of a cheap
// enclosure of RN(u^e) (pow_enclose.h); only where they differ (about one
// evaluation in 10^8, counted) is RN(u^e) itself evaluated, by the
// double-double power (its decisions are those of the two-phase power that
// fills a lattice's table wherever it decides).  That call stays out of line,
// so the kernel holds only the enclosure's registers.
// Segments go in batches of SB: the enclosure runs stage by stage over the
// batch (all its log-table reads, then all its exp-table reads, from copies
// of the tables in LDS), the batch's gathers are issued together, and the
// sums are taken in segment order, as one segment at a time would.  Without
// the batches each segment's chain of dependent reads ran alone.  Sorting the
// list by f0 (the caller's perm) keeps neighbouring lanes on neighbouring
// columns for the gathers.
// ANT: some detector carries antenna-pattern weights.  Without, the kernel
// holds none of their per-detector values, which leaves the scalar registers
// to the power's constants (else they spill into vector-register lanes).
// DOP: every detector has a Doppler table (one sky direction for the whole
// list), read per segment instead of formed per template.
template <int STORE, bool ANT, bool DOP, int SB>
__global__ __launch_bounds__(256) void template_list_kernel(const ListArgs a) {
    __shared__ double2 s_log[128];
    __shared__ double s_exp[256];
    {
        const EncloseTables ct;
        if (threadIdx.x < 128) {
            double r, t;
            ct.log_entry(threadIdx.x, &r, &t);
            s_log[threadIdx.x] = make_double2(r, t);
        }
        s_exp[threadIdx.x] = ct.exp2_entry(threadIdx.x);
        __syncthreads();
    }
    const LdsTables tab{s_log, s_exp};
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = q < a.n;
    // lanes past the list evaluate its first template and discard it; they
    // take no correctly rounded power and count nothing
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
            for (int jb = j0; jb < je; jb += SB) {
                unsigned idx[SB];
                unsigned open = 0;  // bit b: segment jb + b needs RN(u^e) itself
                EncloseSplit sp[SB];
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const double t = uniform_load(D.t, min(jb + b, je - 1));
                    sp[b] = enclose_split(1.0 + div_rn(t - a.t0, T.tau, rtau));
                }
                double ri[SB], ti[SB];
#pragma unroll
                for (int b = 0; b < SB; ++b) tab.log_entry(sp[b].i, &ri[b], &ti[b]);
                EncloseLog lg[SB];
                double x2[SB];
#pragma unroll
                for (int b = 0; b < SB; ++b) lg[b] = enclose_log(e, sp[b], ri[b], ti[b]);
#pragma unroll
                for (int b = 0; b < SB; ++b) x2[b] = tab.exp2_entry(lg[b].j);
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int j = min(jb + b, je - 1);
                    const double Df = doppler<DOP>(D, j, T);
                    const bool before = uniform_load(D.t, j) < a.t0;  // masked: g = 0
                    double glo, ghi;
                    enclose_ends(enclose_value(lg[b], x2[b]), lg[b].y, e, &glo, &ghi);
                    idx[b] = column(D, T, Df, before ? 0.0 : glo);
                    const bool decided = before || (lg[b].ok && column(D, T, Df, ghi) == idx[b]);
                    if (!decided && jb + b < je && live) open |= 1u << b;
                }
                if (open) {
                    for (int b = 0; b < SB; ++b) {
                        if (!((open >> b) & 1u)) continue;
                        const int j = jb + b;
                        const double u = 1.0 + div_rn(uniform_load(D.t, j) - a.t0, T.tau, rtau);
                        const PowSlow px = pow_dd_call(u, e);
                        idx[b] = column(D, T, doppler<DOP>(D, j, T), px.g);
                        atomicAdd(a.exact_count, 1ull);
                        atomicAdd(a.pow_counts + 1, 1ull);
                        if (px.undecided) atomicAdd(a.pow_counts, 1ull);
                    }
                }
                float p[SB];
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    p[b] = jb + b < je ? Store<STORE>::get(rs, (int)idx[b], (jb + b) * D.pitch_bytes, cnt) : 0.0f;
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    if (jb + b >= je) break;
                    const int j = jb + b;
                    float wq = uniform_load(D.wq, j), wv = uniform_load(D.w, j);
                    if (ANT && D.era)  // antenna-pattern weights for this template's sky direction
                        antenna_weights(D.arms, uniform_load(D.era, j), T.sky[0], T.sky[1], T.sky[2], wv,
                                        uniform_load(D.scale, j), wv, wq);
                    sc = __builtin_fmaf(wq, p[b], sc);
                    const bool inb = (idx[b] - 1u) < nb;
                    nin += inb ? 1 : 0;
                    const float wj = inb ? wv : 0.0f;
                    w1c += wj;
                    w2c = __builtin_fmaf(wj, wj, w2c);
                }
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
        hipLaunchKernelGGL((template_list_kernel<STORE, true, false, kListBatch>), grid, dim3(256), 0, st, a);
    else if (dop)
        hipLaunchKernelGGL((template_list_kernel<STORE, false, true, kListBatch>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((template_list_kernel<STORE, false, false, kListBatch>), grid, dim3(256), 0, st, a);
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
