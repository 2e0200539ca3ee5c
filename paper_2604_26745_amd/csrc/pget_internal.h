// Internal structures shared by the HIP kernels and the host runtime of
// libpget.  Not part of the public ABI (include/pget.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pget {

// One wave marches a group of RG consecutive detector bins of one angle;
// its 64 lanes are RG rays x SPL consecutive samples (lane = ray*SPL + sample).
constexpr int RG = 16;
constexpr int SPL = 4;
constexpr int WAVE = 64;
// Pixel tile of the adjoint gather and its lattice footprint per angle.
constexpr int VT = 32;            // tile edge in pixels
constexpr int VFP = 52;           // staged footprint edge in lattice points (>= VT*sqrt2 + 6)
constexpr int VJP_THREADS = 256;  // 4 pixels per thread
constexpr int EW_THREADS = 256;   // element-wise kernels
constexpr int MAX_TAPS = 65;      // 2*32 + 1

// Geometry of one slice shape, as the kernels see it.
struct Geo {
    int n;          // N
    int n_angles;
    int n_bins;
    int n_t;        // samples per ray
    int K;          // collimator half width
    int pitch;      // N + 2: row pitch of the zero-bordered image
    int n_groups;   // ceil(n_bins / RG)
    float step;     // sample spacing
    float bin_size;
    float t_off;    // (n_t - 1) / 2
    float s_off;    // (n_bins - 1) / 2
    float half;     // (N - 1) / 2
    float c_att;    // attenuation scale c
    float kq;       // -c * step^2: weight of the attenuation derivative
    float ln2_scale;  // c * step * log2(e): exponent scale for exp2
    int paired;     // n_angles even over a full turn: angle a + n_angles/2 samples the
                    // same lattice points as angle a with bins and samples mirrored
    int quad;       // paired, n_angles % 4 == 0, step == bin_size and n_bins - n_t even:
                    // sample (i', j') of angle a + n_angles/4 is the point (i, j) =
                    // (rot_c - j', i' + rot_d) of angle a's lattice
    int rot_c;      // (n_t + n_bins)/2 - 1
    int rot_d;      // (n_bins - n_t)/2
};

// Device-resident tables of a plan.
struct Tables {
    const float4* trig;   // [n_angles]: (step*cos, step*sin, cos, sin)
    const float2* rbase;  // [n_angles][n_bins]: (col, row) of the ray at t = 0
    const int2* clip;     // [n_angles][n_bins]: samples [lo, hi] inside the support; lo > hi if none
    const int2* grange;   // [n_angles][n_groups]: union of the group's clip ranges
    const float* taps;    // [2K + 1]
    const int* roff;      // [n_angles][n_bins]: offset of the ray's first in-support sample in the
                          // compacted per-sample arrays (a ray's samples lo..hi contiguous)
    const int2* gcol;     // [n_angles][n_bins]: the adjoint's column table (lo | len << 16,
                          // b = roff - lo; (0, 0) for an empty ray): sample i of the ray sits
                          // at b + i; in paired geometry the mirror ray (range the reflection
                          // of [lo, hi]) is stored right after it, its sample at the same
                          // point at b + 2 hi + 1 - i
    const float* depth;   // [n_t]: depth factor of the attenuation path per sample, or nullptr (1)
    const float* resp;    // [n_t]: weight alpha_i of the far collimator response per sample, or
                          // nullptr (the response is taps at every depth)
    const float* taps_far;  // [2K + 1] with resp: the far response (symmetric)
};

// Per-slice LM parameters on the device.
struct LMParamsDev {
    double alpha_f, alpha_mu, alpha_decay;
    int alpha_decay_until;
    int max_outer, n_cg;
    double beta0, tau, eta, d_f, d_mu;
    double f_lo, f_hi, mu_lo, mu_hi, tol;
    double w_f, w_mu;       // CG preconditioner W = diag(w_f I, w_mu I)
    int active_set;         // 1: CG on the free variables only
    const float* prior_w;   // geometry prior weights (2 N^2, f then mu) or nullptr
    const float* prior_ref; // its reference maps (2 N^2) or nullptr (zero)
    float* trace_u;         // [max_outer][2 N^2]: iterate of each outer iteration, or nullptr
    float* trace_t;         // [max_outer][2 N^2]: its trial point, or nullptr
    int step_sgp;           // 1: the damped step by scaled gradient projection, 0: by CG
    int has_replay;
    int8_t replay[256];
};

// Per-slice LM state on the device.
struct LMState {
    double beta, nu, beta_init;
    double phi_u;        // Phi at the current iterate (with this iteration's alphas)
    double alpha_f, alpha_mu;  // alphas of the current outer iteration
    int k;               // outer iterations done
    int dirty;           // iterate changed since the last linearisation
    int done;            // solve finished (early exit / non-finite)
    int accepted;        // decision of the last outer iteration
    int hook_keep;       // the hook's proposal replaces the LM trial point
    int done_next;       // stop after this iteration's commit
    int final_slot;      // slot holding ||A(u) - y||^2 of the current iterate
    int stop_reason;
    int status;
    double pred, ared, rho;    // of the last LM step
    // scaled gradient projection of the current step: steplength, the
    // alternation threshold, the last Barzilai-Borwein (second rule) values,
    // the line-search factor of the last iteration, and q(s)
    double sgp_alpha, sgp_tau, sgp_bb2[3], sgp_lambda, sgp_q;
    int sgp_nbb;
};

// Reduction slots: each kernel that reduces writes one double per block.
enum Slot {
    SLOT_PHI_DATA_U = 0,   // ||A(u) - y||^2
    SLOT_PHI_REG_U,        // alpha ||grad u||^2 (both blocks)
    SLOT_PHI_DATA_T,       // ||A(u') - y||^2
    SLOT_PHI_REG_T,        // alpha ||grad u'||^2
    SLOT_GS,               // g . s
    SLOT_SRS,              // s . R s
    SLOT_JS,               // ||J s||^2
    SLOT_SNORM,            // ||s||^2
    SLOT_UNORM,            // ||u||^2
    SLOT_GNORM,            // ||g||^2
    SLOT_GAMMA,            // p . q
    SLOT_RR0,              // r.r of CG step m lives in SLOT_RR0 + m % 3: a step reads
    SLOT_RR1,              // the slots of m and m-1 while writing m+1, so three
    SLOT_RR2,              // rotating slots keep readers and writers apart
    SLOT_J1,               // ||J 1||^2 (initial damping)
    SLOT_PHI_DATA_H,       // ||A(u~) - y||^2 of a hook proposal
    SLOT_SGP_GD,           // scaled gradient projection: grad q . d
    SLOT_SGP_DMD,          // d . M d
    SLOT_SGP_N1,           // d . W^-2 d
    SLOT_SGP_D1,           // d . W^-1 M d
    SLOT_SGP_N2,           // d . W M d
    SLOT_SGP_D2,           // (M d) . W^2 (M d)
    N_SLOTS
};
constexpr int SLOT_WIDTH = 1024;   // max blocks per slice of any reducing launch
__host__ __device__ constexpr int rr_slot(int m) { return SLOT_RR0 + (m % 3); }

// Report arrays kept on the device during a solve (per slice).
struct ReportDev {
    double* phi;     // [max_outer + 1]
    double* rho;     // [max_outer]
    double* beta;
    double* pred;
    double* ared;
    double* gnorm;
    int8_t* accepted;
    int8_t* hook_accepted;
    double* cg_rr;   // [max_outer * n_cg]
    double* scalars; // [4]
    double* hook_rho;   // [max_outer]
    double* hook_pred;  // [max_outer]
};


// Source of the map pair staged for an operator: a, a + beta*b (CG search
// direction p = r + beta p_old, beta = rr_m / rr_{m-1}), or all ones.
struct PairSrc {
    const float* af;
    const float* am;
    const float* bf;
    const float* bm;
    long long stride;     // elements between slices
    int kind;             // 0: a; 1: a + beta*b; 2: ones
    int rr_slot_cur;      // kind 1: slots holding r.r of this and the previous CG step
    int rr_slot_prev;
    int n_rr;             // partials per rr slot
    int first;            // kind 1: 1 on the first CG step (beta = 0)
    const LMParamsDev* prm;  // kind 1: per-slice scales w_f, w_mu of a (nullptr: 1)
};

enum MarchMode { MARCH_FWD = 0, MARCH_LIN = 1, MARCH_TRIAL = 2 };
enum JvpMode { JVP_PLAIN = 0, JVP_NORMAL = 1, JVP_SQNORM = 2 };

struct MarchArgs {
    Geo g;
    Tables t;
    PairSrc src;            // (f, mu)
    const void* gimg;       // global bordered image when not staged in LDS
    long long gimg_stride;
    void* wts;              // MARCH_LIN: [n_angles][n_t][n_bins] (step*E, R') pairs
    float* tsum;            // MARCH_LIN: [n_angles][n_bins] sum of lambda*E
    float* wq;              // depth response, MARCH_LIN: R' of the far response, as wts
    long long far_off;      // depth response: elements from a sinogram plane (tsum, wout) to its far plane
    long long wts_stride, sino_stride;
    const float* ymeas;     // measured sinogram (residual modes) or null
    float* yout;            // MARCH_FWD: A(f, mu); MARCH_LIN: optional
    float* wout;            // K (A - y) (MARCH_LIN with ymeas)
    double* part;           // reduction slots
    int slot;               // slot of ||A - y||^2
    const LMState* st;      // skip flags (null: always run)
    int angles_per_block;
};

struct JvpArgs {
    Geo g;
    Tables t;
    PairSrc src;            // the direction v (or the CG direction p)
    const void* gimg;
    long long gimg_stride;
    const void* wts;
    const float* tsum;
    const float* wq;        // depth response: R' of the far response per sample
    long long far_off;      // depth response: far plane of tsum and (NORMAL) out
    long long wts_stride, sino_stride;
    float* out;             // PLAIN: K z;  NORMAL: K K z
    double* part;
    int slot;               // SQNORM: slot of ||K z||^2
    const LMState* st;
    int only_k0;            // initial-damping probe of a slot pool: only slices at iteration 0
    int angles_per_block;   // angle slots per block (a slot is an angle pair when paired)
    int bands;              // staged map in row bands (IMG_BANDS): their count
    int band_h;             // ... and the top bordered rows per band
};

struct VjpArgs {
    Geo g;
    Tables t;
    const void* wts;
    const float* tsum;
    const float* wt;        // blurred cotangent per ray [n_angles][n_bins]
    const float* wq;        // depth response: R' of the far response per sample
    long long far_off;      // depth response: far plane of tsum and wt
    long long wts_stride, sino_stride;
    float* gpart;           // [fine][slices][2][N][N]
    long long gpart_group_stride, gpart_slice_stride;
    int tiles_x;            // ceil(N / VT)
    int groups;             // blocks per tile and slice, each running fpb fine groups
    int fine;               // fine angle groups (fixed by the plan)
    int spf;                // angle slots per fine group
    int fpb;                // fine groups per block: fine <= groups * fpb
    int gs;                 // fine groups per super group (fixed by the plan)
    int super_out;          // 1: a block sums whole super groups and writes one partial
                            // image per super group (fpb a multiple of gs); 0: one per fine group
    const LMState* st;
    int skip_if_clean;
};

struct VecArgs {
    Geo g;
    long long vstride;      // 2 N^2
    float* u;               // current iterate (f, mu)
    float* ut;              // trial iterate
    float* s;               // step u' - u
    float* x;               // CG solution
    float* r;               // CG residual
    float* p;               // CG direction (previous step's on entry to k_cg_x)
    float* q;               // (J^T J + beta D + R) p
    float* grad;            // gradient g
    uint8_t* fmask;         // 1 where a variable is free (active set on)
    const float* gpart;     // group partials of the adjoint
    long long gpart_group_stride, gpart_slice_stride;
    int groups;             // partial images (fine or super groups), summed in order
    int gfold;              // partials per super group: gs for fine partials, 1 for super ones
    double* part;
    int n_ew_blocks;        // partials of element-wise slots
    int n_angle_parts;      // partials of SLOT_JS / J1 / PHI_DATA_* (one per angle)
    LMState* st;
    const LMParamsDev* prm;
    ReportDev* rep;
    int cg_step;            // CG step index m (k_cg_q / k_cg_x / k_jvp source)
    int hook_mode;          // k_trial: 1 -> ut holds the hook's proposal (no clamp)
};

// Storage of the two large streams (staged map pairs, per-sample weight
// pairs): FP32 pairs, or BF16 pairs packed in 32 bits.  Arithmetic is FP32
// either way.
struct F32S;
struct BF16S;
struct F32DR;   // FP32 with a depth-dependent collimator response
template <bool LDS_IMG, int MODE, typename S> __global__ void k_march(MarchArgs A);
// Where k_jvp_lin reads the direction: a bordered copy in HBM, the whole
// bordered pair staged in LDS, or the pair staged in LDS one band of rows at
// a time.
enum { IMG_HBM = 0, IMG_LDS = 1, IMG_BANDS = 2 };
template <int IMG, int MODE, typename S> __global__ void k_jvp_lin(JvpArgs A);
template <typename S>
__global__ void k_pack(Geo g, PairSrc s, const double* part, void* out, long long out_stride,
                       const LMState* st);
__global__ void k_psf(Geo g, const float* taps_g, const float* in, float* out);
template <typename S, bool QUAD> __global__ void k_vjp_lin(VjpArgs A, const float4* trig, const int2* gcol);
__global__ void k_fill_zero(float4* p, long long n4);
__global__ void k_sum_groups(int n2, int groups, int gfold, const float* gpart, long long group_stride,
                             float* gf, float* gm);
__global__ void k_grad_init(VecArgs V);
__global__ void k_cg_q(VecArgs V);
__global__ void k_cg_x(VecArgs V);
__global__ void k_sgp_q(VecArgs V);
__global__ void k_sgp_step(VecArgs V);
__global__ void k_sgp_x(VecArgs V);
__global__ void k_trial(VecArgs V);
__global__ void k_trace(VecArgs V);
__global__ void k_beta0(VecArgs V);
__global__ void k_lm_init(LMState* st, const LMParamsDev* prm, int n_slices);
__global__ void k_decide(VecArgs V, int hook_present);
__global__ void k_hook_decide(VecArgs V);
__global__ void k_accept(VecArgs V);
__global__ void k_final_reg(VecArgs V);
__global__ void k_finish(VecArgs V);
__global__ void k_commit(LMState* st, const LMParamsDev* prm, int n_slices);
__global__ void k_pool_clear(LMState* st, int n_slices);
__global__ void k_pool_release(LMState* st, int slot);
__global__ void k_pool_flags(const LMState* st, int* flags, int n_slices);

}  // namespace pget
