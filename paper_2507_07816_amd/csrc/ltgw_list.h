// Internal interface of the explicit-template evaluation (ltgw_list.hip) for
// the C-ABI layer.  Not part of the public boundary.
#pragma once
#include "ltgw_antenna.h"
#include "ltgw_internal.h"

namespace ltgw {

// One detector as the explicit-template kernel reads it: the store and the
// raw per-segment inputs (the tables of a lattice do not apply: every
// template has its own (tau, n) and sky direction).
struct ListDet {
    const void *store;
    int32_t pitch_bytes;
    int32_t n_seg, n_bins;
    const double *t;  // [n_seg] segment times
    const double *v;  // [n_seg][3] velocities
    const float *wq;  // [n_seg] weights x per-segment scale (the power sum)
    const float *w;   // [n_seg] weights (W1, W2)
    double t_sft, cshift;
    const double *era;     // [n_seg] Earth rotation angles, or NULL: no antenna factor
    const float *scale;    // [n_seg] store row scales (antenna weights are formed per template)
    Arms arms;
    const double *dop;     // [n_seg] Doppler factor 1 + v.n/c when every template has the same sky
                           // direction n (the lattice's table for it), or NULL: formed per template
};

struct ListArgs {
    ListDet det[LTGW_MAX_SEARCH_DET];
    int32_t n_det;
    double t0;
    const ltgw_template *tpl;  // [n] in the caller's order
    const int32_t *perm;       // [n] evaluation order: lane q takes template perm[q]
    int64_t n;
    double *s, *w1, *w2;       // [n] results in the caller's order
    int32_t *c, *n_in;
    float *out_s;              // optional caller outputs
    int32_t *out_c, *out_n;
    unsigned long long *in_band_total;
    unsigned long long *pow_counts;  // [0] undecided powers, [1] powers that took the double-double phase
    unsigned long long *exact_count;  // evaluations whose column the power's enclosure left open
};

hipError_t launch_template_list(int store, const ListArgs &a, hipStream_t st);

}  // namespace ltgw
