// HIP kernels for gfx950 of the PGET Levenberg-Marquardt hot path.
//
// Operators (arXiv 2604.26745, Sec. 2.1, eq. fwd_model / eq. d_fwd_model /
// eq. frechet):
//   k_march     ray march of A(f, mu): bilinear samples of the rotated maps,
//               suffix sum of attenuation toward the detector, exp, ray sum,
//               collimator blur across bins.  In linearising mode it also
//               stores, per lattice sample, step*E_i and the suffix sum R'_i of
//               lambda*E (half of its own term included), from which every
//               Jacobian product of the outer iteration follows without exp.
//   k_jvp_lin   J v from the stored weights: per ray
//               sum_i step*E_i vf_i + kq * (T - R'_i) vmu_i,  T = sum_i lambda_i E_i.
//   k_vjp_lin   J^T w as a gather: for every pixel and angle the (at most 3x3)
//               lattice samples whose bilinear footprint covers the pixel.
// Solver (Sec. 2.2, eqs. m-function, LMA-step; Sec. 3.1, eq. rho_agreement):
//   element-wise CG kernels, trial / model-decrease kernel, decision kernel.
//
// Work mapping: one wavefront = RG consecutive bins (rays) of one angle x
// SPL consecutive samples per ray; lanes of a ray form a DPP quad.  A
// workgroup owns a block of angles and stages the whole zero-bordered map
// pair (interleaved float2) in LDS when it fits; otherwise the maps are read
// from a global bordered copy through the caches.  Reductions are FP64 and
// deterministic: every block writes one partial, consumers sum the partials
// in index order.
#include "pget_internal.h"

#include <math.h>

namespace pget {

// ------------------------------------------------------------------ helpers
template <int CTRL>
__device__ __forceinline__ float qperm(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// quad_perm encodings: lane i of each quad reads lane p_i
constexpr int QP_SHIFT1 = 0 | (0 << 2) | (1 << 4) | (2 << 6);  // [0,0,1,2]
constexpr int QP_SHIFT2 = 0 | (0 << 2) | (0 << 4) | (1 << 6);  // [0,0,0,1]
constexpr int QP_BCAST3 = 3 | (3 << 2) | (3 << 4) | (3 << 6);  // [3,3,3,3]
constexpr int QP_SWAP1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);   // [1,0,3,2]
constexpr int QP_SWAP2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);   // [2,3,0,1]

// inclusive prefix sum over the 4 lanes of a quad (lane order = sample order
// from the detector side), and the quad total
__device__ __forceinline__ void quad_scan(float x, int q, float& incl, float& total)
{
    float s = x;
    float t = qperm<QP_SHIFT1>(s);
    s += (q >= 1) ? t : 0.0f;
    t = qperm<QP_SHIFT2>(s);
    s += (q >= 2) ? t : 0.0f;
    incl = s;
    total = qperm<QP_BCAST3>(s);
}

__device__ __forceinline__ float quad_sum(float x)
{
    x += qperm<QP_SWAP1>(x);
    x += qperm<QP_SWAP2>(x);
    return x;
}

// Sum over the LANES consecutive lanes of one ray (a power of two <= 64),
// returned to all of them: quad permutes, then butterflies across quads.
template <int LANES>
__device__ __forceinline__ float ray_sum(float x)
{
    x += qperm<QP_SWAP1>(x);
    if (LANES >= 4) x += qperm<QP_SWAP2>(x);
#pragma unroll
    for (int o = 4; o < LANES; o <<= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over the block, returned to every thread (fixed order).
__device__ double block_sum(double v, double* sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    __syncthreads();
    return s;
}

// Sum of n partials (one per producing block or angle); every thread of the
// block gets the result.  The first wave adds them (lane l takes l, l + 64,
// ..., then a fixed butterfly), so the order does not depend on the size of
// the consuming block.
__device__ double sum_partials(const double* p, int n, double* sh)
{
    __syncthreads();   // sh may still be read by an earlier call
    if (threadIdx.x < WAVE) {
        double v = 0.0;
        for (int i = threadIdx.x; i < n; i += WAVE) v += p[i];
        v = wave_sum(v);
        if (threadIdx.x == 0) sh[0] = v;
    }
    __syncthreads();
    return sh[0];
}

__device__ __forceinline__ double* slot_ptr(double* part, int slice, int slot)
{
    return part + ((size_t)slice * N_SLOTS + slot) * SLOT_WIDTH;
}
__device__ __forceinline__ const double* slot_ptr(const double* part, int slice, int slot)
{
    return part + ((size_t)slice * N_SLOTS + slot) * SLOT_WIDTH;
}

// ------------------------------------------------------------ storage
__device__ __forceinline__ uint32_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even on the dropped half
    return u >> 16;
}

struct F32S {
    using px_t = float2;
    using w_t = float2;
    static constexpr bool DR = false;     // no depth-dependent collimator response
    static constexpr int VJP_WAVES = 3;   // gather waves per SIMD (register budget 168)
    // Jacobian product: lanes per ray (8 samples x 8 B = 64 B per ray and
    // load), and loads in flight per lane and ray.  Eight rays per wave keep
    // the trip count close to each ray's length.
    static constexpr int JVP_SPL = 8;
    static constexpr int JVP_JU = 8;
    static __device__ __forceinline__ float2 px(px_t v) { return v; }
    static __device__ __forceinline__ px_t to_px(float2 v) { return v; }
    static __device__ __forceinline__ float2 w(w_t v) { return v; }
    static __device__ __forceinline__ w_t to_w(float a, float b) { return make_float2(a, b); }
};

struct BF16S {
    using px_t = uint32_t;   // low half: first value, high half: second value
    using w_t = uint32_t;
    static constexpr bool DR = false;
    static constexpr int VJP_WAVES = 4;   // half the staged weight registers (budget 128)
    static constexpr int JVP_SPL = 8;     // 8 samples x 4 B = 32 B per ray and load
    static constexpr int JVP_JU = 8;
    static __device__ __forceinline__ float2 px(px_t v)
    {
        return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
    }
    static __device__ __forceinline__ px_t to_px(float2 v) { return bf16_rne(v.x) | (bf16_rne(v.y) << 16); }
    static __device__ __forceinline__ float2 w(w_t v) { return px(v); }
    static __device__ __forceinline__ w_t to_w(float a, float b) { return bf16_rne(a) | (bf16_rne(b) << 16); }
};

// FP32 storage with a depth-dependent collimator response: the response to
// sample i is (1 - alpha_i) K + alpha_i K_far.  The per-sample weight pair
// holds (step*E, R'_near) and a second array the far prefix sums R'_far; the
// ray totals and the blurred cotangents come in a near and a far plane.
struct F32DR : F32S {
    static constexpr bool DR = true;
    static constexpr int VJP_WAVES = 2;   // the far sums double the staged registers
    static constexpr int JVP_JU = 2;      // the far sums take the registers of two more trips
};

// Bilinear sample of the zero-bordered interleaved map pair at (col, row)
// in pixel-index coordinates.  Index clamping keeps FP32 rounding at the
// support edge inside the bordered array.
template <typename S>
__device__ __forceinline__ float2 bilerp(const typename S::px_t* __restrict__ img, int pitch, int n,
                                         float col, float row)
{
    float cf = floorf(col), rf = floorf(row);
    int c0 = min(max((int)cf, -1), n - 1);
    int r0 = min(max((int)rf, -1), n - 1);
    float fc = col - (float)c0, fr = row - (float)r0;
    const typename S::px_t* p = img + (r0 + 1) * pitch + (c0 + 1);
    const float2 v00 = S::px(p[0]), v01 = S::px(p[1]), v10 = S::px(p[pitch]), v11 = S::px(p[pitch + 1]);
    float tx = fmaf(fc, v01.x - v00.x, v00.x);
    float ty = fmaf(fc, v01.y - v00.y, v00.y);
    float bx = fmaf(fc, v11.x - v10.x, v10.x);
    float by = fmaf(fc, v11.y - v10.y, v10.y);
    return make_float2(fmaf(fr, bx - tx, tx), fmaf(fr, by - ty, ty));
}

// ------------------------------------------------------------ map sources

__device__ float resolve_beta(const PairSrc& s, const double* part, int slice, double* sh)
{
    if (s.kind != 1 || s.first) return 0.0f;
    double cur = sum_partials(slot_ptr(part, slice, s.rr_slot_cur), s.n_rr, sh);
    double prev = sum_partials(slot_ptr(part, slice, s.rr_slot_prev), s.n_rr, sh);
    return prev > 0.0 ? (float)(cur / prev) : 0.0f;
}

// Scales of a in a source of kind 1 (the CG preconditioner W of the slice).
__device__ __forceinline__ float2 src_scale(const PairSrc& s, int slice)
{
    if (s.kind != 1 || !s.prm) return make_float2(1.0f, 1.0f);
    return make_float2((float)s.prm[slice].w_f, (float)s.prm[slice].w_mu);
}

__device__ __forceinline__ float2 src_value(const PairSrc& s, int slice, int idx, float beta, float2 w)
{
    if (s.kind == 2) return make_float2(1.0f, 1.0f);
    size_t o = (size_t)slice * s.stride + idx;
    float2 v = make_float2(s.af[o], s.am[o]);
    if (s.kind == 1) {
        v.x = fmaf(beta, s.bf[o], w.x * v.x);
        v.y = fmaf(beta, s.bm[o], w.y * v.y);
    }
    return v;
}

// Stage the zero-bordered pair image ((N+2)^2 float2) into `dst`.  Four
// pixels per thread per trip so that their loads are in flight together.
template <typename S>
__device__ void stage_image(typename S::px_t* dst, const PairSrc& s, int slice, int n, int pitch,
                            float beta)
{
    const int total = pitch * pitch;
    const float2 w = src_scale(s, slice);
    constexpr int U = 4;
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            const int rr = idx / pitch - 1, cc = idx - (idx / pitch) * pitch - 1;
            v[u] = make_float2(0.0f, 0.0f);
            if (idx < total && rr >= 0 && rr < n && cc >= 0 && cc < n)
                v[u] = src_value(s, slice, rr * n + cc, beta, w);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) dst[idx] = S::to_px(v[u]);
        }
    }
}

// Bordered rows [r0, r0 + rows) of the map pair (rows past the bordered
// pair are left unwritten; nothing reads them).
template <typename S>
__device__ void stage_rows(typename S::px_t* dst, const PairSrc& s, int slice, int n, int pitch, float beta,
                           int r0, int rows)
{
    const int total = min(rows, pitch - r0) * pitch;
    const float2 w = src_scale(s, slice);
    constexpr int U = 4;
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            const int br = idx / pitch;
            const int rr = r0 + br - 1, cc = idx - br * pitch - 1;
            v[u] = make_float2(0.0f, 0.0f);
            if (idx < total && rr >= 0 && rr < n && cc >= 0 && cc < n)
                v[u] = src_value(s, slice, rr * n + cc, beta, w);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) dst[idx] = S::to_px(v[u]);
        }
    }
}

// Global bordered copy for maps too large for LDS.
template <typename SP>
__global__ void __launch_bounds__(256) k_pack(Geo g, PairSrc s, const double* part, void* out_v,
                                              long long out_stride, const LMState* st)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    if (st && st[slice].done) return;
    float beta = resolve_beta(s, part, slice, sh);
    const float2 w = src_scale(s, slice);
    const int pitch = g.pitch, total = pitch * pitch;
    typename SP::px_t* dst = static_cast<typename SP::px_t*>(out_v) + (size_t)slice * out_stride;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        int rr = idx / pitch - 1, cc = idx - (idx / pitch) * pitch - 1;
        float2 v = make_float2(0.0f, 0.0f);
        if (rr >= 0 && rr < g.n && cc >= 0 && cc < g.n) v = src_value(s, slice, rr * g.n + cc, beta, w);
        dst[idx] = SP::to_px(v);
    }
}

// ------------------------------------------------------ collimator epilogue
// y[j] = sum_k taps[k] * x[j - k + K], zero outside [0, n_bins).
__device__ __forceinline__ float psf_at(const float* x, const float* taps, int K, int nb, int j)
{
    float acc = 0.0f;
    for (int k = -K; k <= K; ++k) {
        int jj = j - k;
        if (jj >= 0 && jj < nb) acc = fmaf(taps[k + K], x[jj], acc);
    }
    return acc;
}

// ------------------------------------------------------------------ march


// Logical work item of workgroup `lin` (linear id) among `total`: the
// hardware places workgroup lin on XCD lin % N_XCD, so XCD x runs items
// [x * per, (x + 1) * per) in order.  The tail beyond a multiple of N_XCD
// keeps its own ids.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_item(int lin, int total)
{
    const int per = total / N_XCD;
    if (lin >= per * N_XCD) return lin;
    return (lin % N_XCD) * per + lin / N_XCD;
}

// The (slice, block of angles) pair of a product or march workgroup: each
// XCD runs a contiguous run of them, so that the blocks of one slice share
// the L2 that holds its staged maps.
__device__ __forceinline__ int2 slice_block()
{
    const int item = xcd_item(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int slice = item / gridDim.x;
    return make_int2(slice, item - slice * gridDim.x);
}

template <bool LDS_IMG, int MODE, typename S>
__global__ void __launch_bounds__(1024) k_march(MarchArgs A)
{
    extern __shared__ float4 smem_raw[];
    __shared__ float taps[MAX_TAPS];
    const Geo& g = A.g;
    const int2 sb = slice_block();
    const int slice = sb.x;
    if (A.st) {
        if (A.st[slice].done) return;
        if (MODE == MARCH_LIN && !A.st[slice].dirty) return;
    }
    // the objective and the linearisation always see the maps in FP32; S only
    // selects the storage of the weights written for the Jacobian products
    using px_t = typename F32S::px_t;
    using w_t = typename S::w_t;
    px_t* simg = reinterpret_cast<px_t*>(smem_raw);
    const int img_elems = LDS_IMG ? g.pitch * g.pitch : 0;
    float* rowp = reinterpret_cast<float*>(simg + img_elems);   // raw ray sums  [n_bins]
    float* rowr = rowp + g.n_bins;                              // residual      [n_bins]
    float* rowpf = rowr + g.n_bins;    // depth response: ray sums seen through the far response
    __shared__ float taps_f[S::DR ? MAX_TAPS : 1];
    for (int k = threadIdx.x; k < 2 * g.K + 1; k += blockDim.x) {
        taps[k] = A.t.taps[k];
        if (S::DR) taps_f[k] = A.t.taps_far[k];
    }
    if (LDS_IMG) stage_image<F32S>(simg, A.src, slice, g.n, g.pitch, 0.0f);
    const px_t* img = LDS_IMG ? simg : static_cast<const px_t*>(A.gimg) + (size_t)slice * A.gimg_stride;
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int q = lane & (SPL - 1), jj = lane >> 2;
    const float hs = 0.5f;
    for (int ab = 0; ab < A.angles_per_block; ++ab) {
        const int a = sb.y * A.angles_per_block + ab;
        if (a >= g.n_angles) break;
        const float4 tr = A.t.trig[a];
        for (int grp = wave; grp < g.n_groups; grp += nwaves) {
            const int j = grp * RG + jj;
            const bool ray_ok = j < g.n_bins;
            int2 cl = make_int2(1, 0);
            float2 rb = make_float2(0.0f, 0.0f);
            long long ray0 = 0;   // compacted index of the ray's sample 0 (its samples lo..hi stored there)
            if (ray_ok) {
                cl = A.t.clip[(size_t)a * g.n_bins + j];
                rb = A.t.rbase[(size_t)a * g.n_bins + j];
                ray0 = (long long)A.t.roff[(size_t)a * g.n_bins + j] - cl.x;
            }
            const int2 gr = A.t.grange[(size_t)a * g.n_groups + grp];
            float carry_mu = 0.0f, carry_le = 0.0f, carry_dle = 0.0f;
            // depth response: the sums split into the parts seen through the
            // near and the far response (lambda E and, for the Jacobian, d lambda E)
            float carry_lf = 0.0f, carry_dn = 0.0f, carry_df = 0.0f;
            const float* depth = A.t.depth;   // per-sample factor of the attenuation path, or none
            // compacted per-sample arrays of the slice: sample i of this ray
            // at ray0 + i (written only inside the ray's support)
            w_t* wsl = nullptr;
            float* qsl = nullptr;
            if (MODE == MARCH_LIN) {
                wsl = static_cast<w_t*>(A.wts) + (size_t)slice * A.wts_stride;
                if (S::DR) qsl = A.wq + (size_t)slice * A.wts_stride;
            }
            for (int i0 = gr.y; i0 >= gr.x; i0 -= SPL) {
                const int i = i0 - q;
                const bool act = (i >= cl.x) && (i <= cl.y);
                float lam = 0.0f, mu = 0.0f;
                if (act) {
                    const float ti = (float)i - g.t_off;
                    const float col = fmaf(ti, tr.x, rb.x), row = fmaf(ti, tr.y, rb.y);
                    const float2 v = bilerp<F32S>(img, g.pitch, g.n, col, row);
                    lam = v.x;
                    mu = v.y;
                }
                float incl, tot;
                quad_scan(mu, q, incl, tot);
                // B_i / step = carry + (samples nearer the detector) + mu_i / 2
                const float bsum = carry_mu + (incl - hs * mu);
                carry_mu += tot;
                float lincl, ltot;
                if (S::DR) {
                    // carry_le holds the near part; sample i splits lambda E
                    // into (1 - alpha_i) and alpha_i shares
                    const float d = (depth && act) ? depth[i] : 1.0f;
                    const float al = act ? A.t.resp[i] : 0.0f;
                    const float E = __builtin_amdgcn_exp2f(-g.ln2_scale * (d * bsum));
                    const float le = lam * E;
                    const float ln = (1.0f - al) * le, lf = al * le;
                    float fincl, ftot;
                    quad_scan(ln, q, lincl, ltot);
                    quad_scan(lf, q, fincl, ftot);
                    // the Jacobian's sums of d lambda E equal these without a depth factor
                    float dn = ln, dfv = lf, dnincl = lincl, dntot = ltot, dfincl = fincl, dftot = ftot;
                    if (depth) {
                        dn = d * ln;
                        dfv = d * lf;
                        quad_scan(dn, q, dnincl, dntot);
                        quad_scan(dfv, q, dfincl, dftot);
                    }
                    if (MODE == MARCH_LIN && act) {
                        wsl[ray0 + i] = S::to_w(g.step * E, carry_dn + (dnincl - hs * dn));
                        qsl[ray0 + i] = carry_df + (dfincl - hs * dfv);
                    }
                    carry_lf += ftot;
                    carry_dn += dntot;
                    carry_df += dftot;
                } else if (!depth) {
                    const float E = __builtin_amdgcn_exp2f(-g.ln2_scale * bsum);
                    const float le = lam * E;
                    quad_scan(le, q, lincl, ltot);
                    if (MODE == MARCH_LIN && act) {
                        const float rprime = carry_le + (lincl - hs * le);
                        wsl[ray0 + i] = S::to_w(g.step * E, rprime);
                    }
                } else {
                    // E_i = exp(-c d_i B_i); the ray sum needs lam E, the
                    // attenuation part of the Jacobian the sums of d lam E
                    const float d = act ? depth[i] : 1.0f;
                    const float E = __builtin_amdgcn_exp2f(-g.ln2_scale * (d * bsum));
                    const float le = lam * E, dle = d * le;
                    quad_scan(le, q, lincl, ltot);
                    float dincl, dtot;
                    quad_scan(dle, q, dincl, dtot);
                    if (MODE == MARCH_LIN && act) {
                        const float rprime = carry_dle + (dincl - hs * dle);
                        wsl[ray0 + i] = S::to_w(g.step * E, rprime);
                    }
                    carry_dle += dtot;
                }
                carry_le += ltot;
            }
            if (ray_ok && q == 0) {
                rowp[j] = g.step * carry_le;
                const size_t o = (size_t)slice * A.sino_stride + (size_t)a * g.n_bins + j;
                if (S::DR) {
                    rowpf[j] = g.step * carry_lf;
                    if (MODE == MARCH_LIN) {
                        A.tsum[o] = carry_dn;
                        A.tsum[o + A.far_off] = carry_df;
                    }
                } else if (MODE == MARCH_LIN) {
                    A.tsum[o] = depth ? carry_dle : carry_le;
                }
            }
        }
        __syncthreads();
        // collimator blur and epilogue over the bins of this angle
        const size_t srow = (size_t)slice * A.sino_stride + (size_t)a * g.n_bins;
        for (int j = threadIdx.x; j < g.n_bins; j += blockDim.x) {
            float y = psf_at(rowp, taps, g.K, g.n_bins, j);
            if (S::DR) y += psf_at(rowpf, taps_f, g.K, g.n_bins, j);
            if (A.yout) A.yout[srow + j] = y;
            if (A.ymeas) rowr[j] = y - A.ymeas[srow + j];
        }
        if (A.ymeas) {
            __syncthreads();
            // the transposed blurs; both responses are symmetric
            if (A.wout)
                for (int j = threadIdx.x; j < g.n_bins; j += blockDim.x) {
                    A.wout[srow + j] = psf_at(rowr, taps, g.K, g.n_bins, j);
                    if (S::DR) A.wout[srow + A.far_off + j] = psf_at(rowr, taps_f, g.K, g.n_bins, j);
                }
            // ||A - y||^2 of this angle, one partial per angle in a fixed
            // order (the same whatever the angles per block)
            if (A.part && wave == 0) {
                double v = 0.0;
                for (int j = lane; j < g.n_bins; j += WAVE) {
                    const double r = rowr[j];
                    v += r * r;
                }
                v = wave_sum(v);
                if (lane == 0) slot_ptr(A.part, slice, A.slot)[a] = v;
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- linear JVP


// Work items of a block are (angle slot, ray group) pairs spread over all
// waves; one barrier precedes the collimator epilogue of every angle of the
// block.  When the geometry is paired, a slot holds angle a and its mirror
// a' = a + n_angles/2: ray j of a and ray n_bins-1-j of a' visit the same
// points (sample i of one is sample n_t-1-i of the other), so one bilinear
// sample of the direction serves both rays.
//
// Maps whose bordered pair does not fit in LDS are walked in the plan's
// bands of rows (A.bands > 1): the block runs its items once per band, each
// sample in the band that holds its bilinear footprint's top row, and a
// ray's partial sums are added to its row value in band order.  IMG_BANDS
// stages each band in LDS; IMG_HBM reads the same samples from the bordered
// copy in the same order, so the two give the same bits and the choice
// between them (by the block's angle slots) is a launch shape only.
template <int IMG, int MODE, typename S>
__global__ void __launch_bounds__(1024) k_jvp_lin(JvpArgs A)
{
    constexpr bool LDS_IMG = IMG != IMG_HBM;
    constexpr bool STAGE_BANDS = IMG == IMG_BANDS;
    // The band walk: always when staging bands (bands outside the items: each
    // band staged once per block), never with the whole pair in LDS, and
    // from the HBM copy when the plan has bands (bands inside each item: its
    // set-up done once, the per-band values added in band order in
    // registers).  Block-uniform.
    const bool INNER = IMG == IMG_HBM && A.bands > 1;
    const bool BANDS = STAGE_BANDS || INNER;
    extern __shared__ float4 smem_raw[];
    __shared__ double sh[16];
    __shared__ float taps[MAX_TAPS];
    const Geo& g = A.g;
    const int2 sb = slice_block();
    const int slice = sb.x;
    if (A.st && A.st[slice].done) return;
    if (A.only_k0 && A.st && A.st[slice].k != 0) return;   // initial-damping probe of a slot pool
    const int per_slot = g.paired ? 2 : 1;
    const int n_slots = g.paired ? g.n_angles / 2 : g.n_angles;
    const int slot0 = sb.y * A.angles_per_block;
    const int nslot = min(A.angles_per_block, n_slots - slot0);
    const int nrows = nslot * per_slot;   // sinogram rows produced by this block
    using px_t = typename S::px_t;
    using w_t = typename S::w_t;
    px_t* simg = reinterpret_cast<px_t*>(smem_raw);
    const int img_elems = LDS_IMG ? (STAGE_BANDS ? (A.band_h + 1) * g.pitch : g.pitch * g.pitch) : 0;
    float* rowz = reinterpret_cast<float*>(simg + img_elems);   // [nrows][n_bins]
    float* rowy = rowz + A.angles_per_block * per_slot * g.n_bins;
    float* rowzf = rowy + A.angles_per_block * per_slot * g.n_bins;   // depth response: far part of z
    float* alpha = rowzf + A.angles_per_block * per_slot * g.n_bins;  // depth response: alpha per sample
    __shared__ float taps_f[S::DR ? MAX_TAPS : 1];
    for (int k = threadIdx.x; k < 2 * g.K + 1; k += blockDim.x) {
        taps[k] = A.t.taps[k];
        if (S::DR) taps_f[k] = A.t.taps_far[k];
    }
    if (S::DR)
        for (int i = threadIdx.x; i < g.n_t; i += blockDim.x) alpha[i] = A.t.resp[i];
    const float beta = LDS_IMG ? resolve_beta(A.src, A.part, slice, sh) : 0.0f;

    // A wave covers JR consecutive rays with JSPL lanes per ray; the weights
    // of a ray's in-support samples are contiguous (compacted arrays), so one
    // load instruction reads JSPL consecutive samples of each of its rays.
    // The mirror ray holds the same points in reverse order (sample i of this
    // ray is sample n_t - 1 - i of the mirror), stored right after the ray.
    constexpr int JSPL = S::JVP_SPL;
    constexpr int JR = 64 / JSPL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int q = lane & (JSPL - 1), jj = lane / JSPL;
    const w_t* wslice = static_cast<const w_t*>(A.wts) + (size_t)slice * A.wts_stride;
    const float* qslice = S::DR ? A.wq + (size_t)slice * A.wts_stride : nullptr;
    const float* tslice = A.tsum + (size_t)slice * A.sino_stride;
    // Items are taken from a block-wide counter (dynamic balance), longest
    // first: ray groups ordered from the middle of the detector outward.
    __shared__ int next_item;
    const int n_ig = (g.n_bins + JR - 1) / JR;
    const int n_items = nslot * n_ig;
    const int gc = n_ig / 2;
    const int n_outer = STAGE_BANDS ? A.bands : 1;
    const int n_inner = INNER ? A.bands : 1;
    for (int band = 0; band < n_outer; ++band) {
    // top bordered rows [SB0, ...) of the staged band
    const int SB0 = STAGE_BANDS ? band * A.band_h : 0;
    // every wave is done with the previous band's items (their counter is
    // reset below) and its staged rows
    if (STAGE_BANDS && band > 0) __syncthreads();
    if (LDS_IMG) {
        if (STAGE_BANDS) stage_rows<S>(simg, A.src, slice, g.n, g.pitch, beta, SB0, A.band_h + 1);
        else stage_image<S>(simg, A.src, slice, g.n, g.pitch, beta);
    }
    // bordered row r of the map pair at img[r * pitch]
    const px_t* img = LDS_IMG ? simg - (STAGE_BANDS ? (ptrdiff_t)SB0 * g.pitch : 0)
                              : static_cast<const px_t*>(A.gimg) + (size_t)slice * A.gimg_stride;
    if (threadIdx.x == 0) next_item = nwaves;
    __syncthreads();
    for (int item = wave; item < n_items;) {
        const int rank = item / nslot, sl = item - rank * nslot;
        const int grp = (rank & 1) ? gc - (rank + 1) / 2 : gc + rank / 2;
        const int a = slot0 + sl;
        const int am = a + g.n_angles / 2;   // mirror angle (paired only)
        const float4 tr = A.t.trig[a];
        const int j = grp * JR + jj;
        const int jm = g.n_bins - 1 - j;
        const bool ray_ok = j < g.n_bins;
        int2 cl = make_int2(1, 0), clm = make_int2(1, 0);
        float2 rb = make_float2(0.0f, 0.0f);
        float T = 0.0f, Tm = 0.0f, Tf = 0.0f, Tfm = 0.0f;
        long long off = 0, offm = 0;   // compacted index of the ray's first in-support sample
        if (ray_ok) {
            cl = A.t.clip[(size_t)a * g.n_bins + j];
            rb = A.t.rbase[(size_t)a * g.n_bins + j];
            off = A.t.roff[(size_t)a * g.n_bins + j];
            T = tslice[(size_t)a * g.n_bins + j];
            if (g.paired) {
                clm = A.t.clip[(size_t)am * g.n_bins + jm];
                offm = A.t.roff[(size_t)am * g.n_bins + jm];
                Tm = tslice[(size_t)am * g.n_bins + jm];
            }
            if (S::DR) {
                Tf = tslice[A.far_off + (size_t)a * g.n_bins + j];
                if (g.paired) Tfm = tslice[A.far_off + (size_t)am * g.n_bins + jm];
            }
        }
        const int len = cl.y - cl.x + 1;   // <= 0 without support
        // with bands inside the item: the running sum of its per-band values
        float tz = 0.0f, tzm = 0.0f, tzf = 0.0f, tzfm = 0.0f;
        for (int ib = 0; ib < n_inner; ++ib) {
        // top bordered rows [B0, B1) of this pass's samples
        const int bidx = STAGE_BANDS ? band : ib;
        const int B0 = BANDS ? bidx * A.band_h : 0;
        const int B1 = BANDS ? min(B0 + A.band_h, g.n + 1) : g.n + 1;
        // The ray's samples this pass visits: all of its support, or with
        // bands a superset of those whose top bilinear row lies in [B0, B1)
        // (from the row's slope along the ray, two samples of margin; rays
        // nearly along the rows keep them all), tested exactly per sample.
        int c_lo = 0, c_hi = len;
        if (BANDS && len > 0 && fabsf(tr.y) >= 0.01f) {
            const float base = (float)cl.x - g.t_off;
            const float ca = ((float)(B0 - 1) - rb.y) / tr.y - base;
            const float cb = ((float)(B1 - 1) - rb.y) / tr.y - base;
            const float lo_f = fminf(fmaxf(fminf(ca, cb), -4.0f), (float)len + 4.0f);
            const float hi_f = fminf(fmaxf(fmaxf(ca, cb), -4.0f), (float)len + 4.0f);
            c_lo = max(0, (int)floorf(lo_f) - 2);
            c_hi = min(len, (int)ceilf(hi_f) + 2);
        }
        // trips of the item: from the first to the last sample any of its
        // rays visits (wave-uniform; without bands from 0 to the longest ray)
        int tlo = 0, tmax = len;
        if (BANDS) {
            const bool any = len > 0 && c_hi > c_lo;
            tlo = any ? c_lo : 0x3fffffff;
            tmax = any ? c_hi : 0;
#pragma unroll
            for (int o = JSPL; o < 64; o <<= 1) tlo = min(tlo, __shfl_xor(tlo, o, 64));
            // from a multiple of JSPL: sample c on lane c mod JSPL in every
            // band and launch shape
            tlo = __builtin_amdgcn_readfirstlane(tlo) / JSPL * JSPL;
        }
#pragma unroll
        for (int o = JSPL; o < 64; o <<= 1) tmax = max(tmax, __shfl_xor(tmax, o, 64));
        tmax = __builtin_amdgcn_readfirstlane(tmax);
        // sample c in this pass's band (the top row as the bilinear lookup
        // computes it)
        auto in_band = [&](int c) -> bool {
            if (!BANDS) return true;
            const float row = fmaf((float)(cl.x + c) - g.t_off, tr.y, rb.y);
            const int rt = min(max((int)floorf(row), -1), g.n - 1) + 1;
            return rt >= B0 && rt < B1;
        };
        float accf = 0.0f, accq = 0.0f, accfm = 0.0f, accqm = 0.0f;
        // depth response: accf / accq collect the near parts, these the far
        float accff = 0.0f, accqf = 0.0f, accffm = 0.0f, accqfm = 0.0f;
        // The sample loop is software-pipelined: the weights of trip t+1 (JU
        // samples per lane) are loaded while trip t is computed; they stay in
        // their storage format until used.  Lanes past their ray's support
        // load nothing and use (0, T), which makes both terms vanish.  Sample
        // c of the trip pattern is the ray's sample lo + c; the mirror holds it
        // at its own sample n_t - 1 - i (inside the mirror's support, which
        // equals this ray's reversed).
        constexpr int JU = S::JVP_JU;
        constexpr int STEP = JU * JSPL;
        constexpr int QU = S::DR ? JU : 1;
        w_t wa[JU], wma[JU], wb[JU], wmb[JU];
        float qa[QU], qma[QU], qb[QU], qmb[QU];
        // sub-steps past the item's longest ray are skipped (wave-uniform)
        auto load = [&](int c0, w_t* w, w_t* wm, float* qv, float* qm) {
#pragma unroll
            for (int u = 0; u < JU; ++u) {
                if (u > 0 && c0 + u * JSPL >= tmax) break;
                const int c = c0 + u * JSPL + q;
                const bool ok = c < len && in_band(c);
                const int i = cl.x + c;
                const long long cm = (long long)(g.n_t - 1 - i - clm.x);
                w[u] = ok ? wslice[off + c] : w_t{};
                if (g.paired) wm[u] = ok ? wslice[offm + cm] : w_t{};
                if constexpr (S::DR) {
                    qv[u] = ok ? qslice[off + c] : 0.0f;
                    if (g.paired) qm[u] = ok ? qslice[offm + cm] : 0.0f;
                }
            }
        };
        auto compute = [&](int c0, const w_t* w, const w_t* wm, const float* qv, const float* qm) {
#pragma unroll
            for (int u = 0; u < JU; ++u) {
                if (u > 0 && c0 + u * JSPL >= tmax) break;
                const int c = c0 + u * JSPL + q;
                const bool ok = c < len && in_band(c);
                const int i = cl.x + c;
                const float ti = (float)i - g.t_off;
                const float col = fmaf(ti, tr.x, rb.x), row = fmaf(ti, tr.y, rb.y);
                // with bands, lanes whose sample is not in this band look up a
                // row of the band (their value is discarded)
                const float2 v = bilerp<S>(img, g.pitch, g.n, col, (BANDS && !ok) ? (float)B0 - 0.5f : row);
                const float2 wv = S::w(w[u]);
                if constexpr (S::DR) {
                    const float al = ok ? alpha[i] : 0.0f;
                    const float ef = wv.x * v.x;
                    accf = fmaf(1.0f - al, ef, accf);
                    accff = fmaf(al, ef, accff);
                    accq = fmaf(T - (ok ? wv.y : T), v.y, accq);
                    accqf = fmaf(Tf - (ok ? qv[u] : Tf), v.y, accqf);
                    if (g.paired) {
                        const float2 wmv = S::w(wm[u]);
                        const float alm = ok ? alpha[g.n_t - 1 - i] : 0.0f;
                        const float efm = wmv.x * v.x;
                        accfm = fmaf(1.0f - alm, efm, accfm);
                        accffm = fmaf(alm, efm, accffm);
                        accqm = fmaf(Tm - (ok ? wmv.y : Tm), v.y, accqm);
                        accqfm = fmaf(Tfm - (ok ? qm[u] : Tfm), v.y, accqfm);
                    }
                } else {
                    accf = fmaf(wv.x, v.x, accf);
                    accq = fmaf(T - (ok ? wv.y : T), v.y, accq);
                    if (g.paired) {
                        const float2 wmv = S::w(wm[u]);
                        accfm = fmaf(wmv.x, v.x, accfm);
                        accqm = fmaf(Tm - (ok ? wmv.y : Tm), v.y, accqm);
                    }
                }
            }
        };
        int c0 = tlo;
        if (c0 < tmax) load(c0, wa, wma, qa, qma);
        while (c0 < tmax) {
            const int c1 = c0 + STEP;
            if (c1 < tmax) load(c1, wb, wmb, qb, qmb);
            compute(c0, wa, wma, qa, qma);
            if (c1 >= tmax) break;
            const int c2 = c1 + STEP;
            if (c2 < tmax) load(c2, wa, wma, qa, qma);
            compute(c1, wb, wmb, qb, qmb);
            c0 = c2;
        }
        // a ray's value: this pass's sum, added in band order with bands
        // (in the row value when the bands are staged, in registers when
        // they run inside the item: the same additions)
        auto put = [&](float* dst, float& tot, float v) {
            if (INNER) tot = ib > 0 ? tot + v : v;
            else if (ray_ok && q == 0) *dst = (STAGE_BANDS && band > 0) ? *dst + v : v;
        };
        accf = ray_sum<JSPL>(accf);
        accq = ray_sum<JSPL>(accq);
        put(&rowz[sl * g.n_bins + j], tz, fmaf(g.kq, accq, accf));
        if (S::DR) {
            accff = ray_sum<JSPL>(accff);
            accqf = ray_sum<JSPL>(accqf);
            put(&rowzf[sl * g.n_bins + j], tzf, fmaf(g.kq, accqf, accff));
        }
        if (g.paired) {
            accfm = ray_sum<JSPL>(accfm);
            accqm = ray_sum<JSPL>(accqm);
            put(&rowz[(nslot + sl) * g.n_bins + jm], tzm, fmaf(g.kq, accqm, accfm));
            if (S::DR) {
                accffm = ray_sum<JSPL>(accffm);
                accqfm = ray_sum<JSPL>(accqfm);
                put(&rowzf[(nslot + sl) * g.n_bins + jm], tzfm, fmaf(g.kq, accqfm, accffm));
            }
        }
        }   // bands inside the item
        if (INNER && ray_ok && q == 0) {
            rowz[sl * g.n_bins + j] = tz;
            if (S::DR) rowzf[sl * g.n_bins + j] = tzf;
            if (g.paired) {
                rowz[(nslot + sl) * g.n_bins + jm] = tzm;
                if (S::DR) rowzf[(nslot + sl) * g.n_bins + jm] = tzfm;
            }
        }
        int nxt = 0;
        if (lane == 0) nxt = atomicAdd(&next_item, 1);
        item = __shfl(nxt, 0, 64);
    }
    }   // bands
    __syncthreads();
    // collimator epilogue over every (row, bin) of the block; row r < nslot is
    // angle slot0 + r, row nslot + r its mirror
    const int nel = nrows * g.n_bins;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int r = e / g.n_bins, jb = e - r * g.n_bins;
        float y = psf_at(rowz + r * g.n_bins, taps, g.K, g.n_bins, jb);
        if (S::DR) y += psf_at(rowzf + r * g.n_bins, taps_f, g.K, g.n_bins, jb);
        const int a = r < nslot ? slot0 + r : slot0 + (r - nslot) + g.n_angles / 2;
        const size_t o = (size_t)slice * A.sino_stride + (size_t)a * g.n_bins + jb;
        if (MODE == JVP_PLAIN) A.out[o] = y;
        if (MODE != JVP_PLAIN) rowy[e] = y;
    }
    if (MODE == JVP_NORMAL) {
        __syncthreads();
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            const int r = e / g.n_bins, jb = e - r * g.n_bins;
            const int a = r < nslot ? slot0 + r : slot0 + (r - nslot) + g.n_angles / 2;
            const size_t o = (size_t)slice * A.sino_stride + (size_t)a * g.n_bins + jb;
            A.out[o] = psf_at(rowy + r * g.n_bins, taps, g.K, g.n_bins, jb);
            if (S::DR) A.out[o + A.far_off] = psf_at(rowy + r * g.n_bins, taps_f, g.K, g.n_bins, jb);
        }
    }
    if (MODE == JVP_SQNORM) {
        // ||K z||^2 per angle: row r by wave r mod nwaves, in a fixed order
        // (the same whatever the angle slots per block)
        __syncthreads();
        for (int r = wave; r < nrows; r += nwaves) {
            const int a = r < nslot ? slot0 + r : slot0 + (r - nslot) + g.n_angles / 2;
            double v = 0.0;
            for (int jb = lane; jb < g.n_bins; jb += WAVE) {
                const double y = rowy[r * g.n_bins + jb];
                v += y * y;
            }
            v = wave_sum(v);
            if (lane == 0) slot_ptr(A.part, slice, A.slot)[a] = v;
        }
    }
}

// ---------------------------------------------------------- blur of a sinogram
__global__ void __launch_bounds__(256) k_psf(Geo g, const float* taps_g, const float* in, float* out)
{
    __shared__ float taps[MAX_TAPS];
    extern __shared__ float row[];
    const int a = blockIdx.x;
    for (int k = threadIdx.x; k < 2 * g.K + 1; k += blockDim.x) taps[k] = taps_g[k];
    for (int j = threadIdx.x; j < g.n_bins; j += blockDim.x) row[j] = in[(size_t)a * g.n_bins + j];
    __syncthreads();
    for (int j = threadIdx.x; j < g.n_bins; j += blockDim.x)
        out[(size_t)a * g.n_bins + j] = psf_at(row, taps, g.K, g.n_bins, j);
}

// ------------------------------------------------------- adjoint (gather)

// Lattice window of one pixel tile at one angle: first candidate rows/columns
// minus a margin of one, and the window extent (<= VFP).
struct Window {
    int jlo, ilo, wj, wi;
};

__device__ __forceinline__ Window tile_window(const Geo& g, float4 tr, int tr0, int tc0)
{
    const float SQ2 = 1.41421356f;
    const float cs = tr.z, sn = tr.w;
    const float inv_ds = 1.0f / g.bin_size, inv_dt = 1.0f / g.step;
    const float xa = (float)tc0 - g.half, xb = (float)(tc0 + VT - 1) - g.half;
    const float ya = (float)tr0 - g.half, yb = (float)(tr0 + VT - 1) - g.half;
    float umin = 1e30f, umax = -1e30f, vmin = 1e30f, vmax = -1e30f;
#pragma unroll
    for (int cnr = 0; cnr < 4; ++cnr) {
        const float x = (cnr & 1) ? xb : xa, y = (cnr & 2) ? yb : ya;
        const float u = fmaf(-x * sn + y * cs, inv_ds, g.s_off);
        const float v = fmaf(x * cs + y * sn, inv_dt, g.t_off);
        umin = fminf(umin, u); umax = fmaxf(umax, u);
        vmin = fminf(vmin, v); vmax = fmaxf(vmax, v);
    }
    Window w;
    w.jlo = (int)floorf(umin - SQ2);          // first candidate - 1
    w.ilo = (int)floorf(vmin - SQ2);
    // last candidate is floor(max - sqrt2) + 3; one more column of margin
    w.wj = min(VFP, (int)floorf(umax - SQ2) + 5 - w.jlo);
    w.wi = min(VFP, (int)floorf(vmax - SQ2) + 5 - w.ilo);
    // wave-uniform: held in scalar registers
    w.jlo = __builtin_amdgcn_readfirstlane(w.jlo);
    w.ilo = __builtin_amdgcn_readfirstlane(w.ilo);
    w.wj = __builtin_amdgcn_readfirstlane(w.wj);
    w.wi = __builtin_amdgcn_readfirstlane(w.wi);
    return w;
}

// Window of angle a + n_angles/4 holding the same points as window W of
// angle a (quarter-turn geometry): point (i, j) of a is (j - rot_d, rot_c - i)
// of the rotated angle, so the rotated window's columns run over W's rows
// (reversed) and its rows over W's columns.
__device__ __forceinline__ Window rot_window(const Geo& g, const Window& W)
{
    Window r;
    r.jlo = g.rot_c - (W.ilo + W.wi - 1);
    r.ilo = W.jlo - g.rot_d;
    r.wj = W.wi;
    r.wi = W.wj;
    return r;
}

// Window columns per wave: the block's 4 waves take columns (rays) w, w+4,
// ...; lane = window row (sample).  A ray's in-support samples are
// contiguous in the compacted per-sample arrays, so each load reads
// consecutive samples of one ray.
constexpr int VCOLS = (VFP + 3) / 4;
// LDS row pitch of the staged window (odd in float2 pairs' halves: the
// transposed adds of the rotated angles spread over the banks)
constexpr int LP = VFP + 1;

// One angle's window in registers: the weight pair of every point (row
// lane, columns wave + 4k) with the mirror angle's at the same points, and,
// for the LDS column table, the blurred cotangent and ray total of the
// lane's column (lane = column there) and its mirror's.  The weights stay
// in their storage format until they are staged in LDS, so that no
// conversion waits on a load while the previous angle is gathered.
template <typename SP>
struct Stage {
    typename SP::w_t w[VCOLS];
    typename SP::w_t wm[VCOLS];   // mirror angle, same points (paired geometry)
    float4 cv;                    // (wt, T, wt of the mirror, T of the mirror) of column `lane`
    // depth response: R' of the far response per point, the far planes of
    // the column values, and alpha of row `lane` for the angle and its mirror
    static constexpr int QR = SP::DR ? VCOLS : 1;
    float q[QR], qm[QR];
    float4 cvf;
    float al, alm;
    // column table (lo | len << 16, base) of the next angle this stage loads
    // (lane = column): read one angle ahead, so that the weight loads never
    // wait on a dependent load
    int2 ct;
};

// Column-table entries of angle a for window W's columns (lane = column);
// columns off the window or the detector read as empty rays.
__device__ __forceinline__ int2 col_table(const Geo& g, const int2* __restrict__ gcol, int a, const Window& W)
{
    const int lane = threadIdx.x & 63;
    const int j = W.jlo + lane;
    return (lane < W.wj && j >= 0 && j < g.n_bins) ? gcol[(size_t)a * g.n_bins + j] : make_int2(0, 0);
}

// The weights of one window column (rows = lanes) of a stage: zero, then,
// where row i lies in the ray's support [lo, lo + len), the sample and (PAIRED)
// the mirror ray's sample at the same point.  b: element offset of the ray's
// sample 0 (negative when the ray's first sample opens the array), bm: of
// the mirror's sample at sample 0's point (the mirror's range is the
// reflection of the ray's, its samples stored right after it, so its sample
// at row i sits at b + 2 hi + 1 - i).  Byte offsets are formed in 32-bit
// unsigned arithmetic, modulo 2^32: b + i and bm - i lie in [0, 2^29), so
// (b + i) * size is exact whatever the sign of b; iw = i * sizeof(w_t),
// iq = 4 i.
template <typename SP, bool PAIRED>
__device__ __forceinline__ void stage_column(Stage<SP>& S, int k, const char* wb, const char* qb, int i, int lo,
                                             unsigned len, unsigned b, unsigned bm, unsigned iw, unsigned iq)
{
    using w_t = typename SP::w_t;
    constexpr unsigned WB = sizeof(w_t);
    S.w[k] = w_t{};                 // zero in either format
    if (PAIRED) S.wm[k] = w_t{};
    if constexpr (SP::DR) {
        S.q[k] = 0.0f;
        if (PAIRED) S.qm[k] = 0.0f;
    }
    if ((unsigned)(i - lo) < len) {
        S.w[k] = *reinterpret_cast<const w_t*>(wb + (b * WB + iw));
        if (PAIRED) S.wm[k] = *reinterpret_cast<const w_t*>(wb + (bm * WB - iw));
        if constexpr (SP::DR) {
            S.q[k] = *reinterpret_cast<const float*>(qb + (b * 4u + iq));
            if (PAIRED) S.qm[k] = *reinterpret_cast<const float*>(qb + (bm * 4u - iq));
        }
    }
}

// Loads of one angle's window into registers, by the column table read by
// the previous call (S.ct); then reads the table of angle `an` over window
// Wnx for the next call (has_next).  Rows outside a column's support and
// columns off the window or the detector stage zero weights; rows past the
// window (lanes >= W.wi) stage their points' true weights, which the gather
// meets only with a tent weight of exactly zero.
template <typename SP>
__device__ __forceinline__ void stage_load(Stage<SP>& S, const VjpArgs& A, const typename SP::w_t* wbase,
                                           const float* qbase, int slice, int a, const Window& W, bool has_next,
                                           int an, const Window& Wnx, const int2* __restrict__ gcol)
{
    const Geo& g = A.g;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int am = a + g.n_angles / 2;
    const size_t sbase = (size_t)slice * A.sino_stride + (size_t)a * g.n_bins;
    const size_t sbasem = (size_t)slice * A.sino_stride + (size_t)am * g.n_bins;
    const int2 cur = S.ct;
    // column values (lane = column)
    {
        const int j = W.jlo + lane;
        const int jm = g.n_bins - 1 - j;
        const bool jok = lane < W.wj && j >= 0 && j < g.n_bins;
        S.cv = make_float4(jok ? A.wt[sbase + j] : 0.0f, jok ? A.tsum[sbase + j] : 0.0f,
                           (jok && g.paired) ? A.wt[sbasem + jm] : 0.0f,
                           (jok && g.paired) ? A.tsum[sbasem + jm] : 0.0f);
        if constexpr (SP::DR)
            S.cvf = make_float4(jok ? A.wt[A.far_off + sbase + j] : 0.0f, jok ? A.tsum[A.far_off + sbase + j] : 0.0f,
                                (jok && g.paired) ? A.wt[A.far_off + sbasem + jm] : 0.0f,
                                (jok && g.paired) ? A.tsum[A.far_off + sbasem + jm] : 0.0f);
    }
    // weights (lane = row, sample i)
    const int i = W.ilo + lane;
    if constexpr (SP::DR) {
        // sample i of the angle is sample n_t - 1 - i of its mirror; rows off
        // the lattice hold zero weights, any alpha serves them
        const int ic = min(max(i, 0), g.n_t - 1);
        S.al = A.t.resp[ic];
        S.alm = A.t.resp[g.n_t - 1 - ic];
    }
    const char* wb = reinterpret_cast<const char*>(wbase);
    const char* qb = reinterpret_cast<const char*>(qbase);
    const unsigned iw = (unsigned)i * (unsigned)sizeof(typename SP::w_t), iq = (unsigned)i * 4u;
    // entry (lo | len << 16, b): sample i of the ray at b + i
#define PGET_STAGE_COLUMNS(PAIRED)                                                              \
    _Pragma("unroll") for (int k = 0; k < VCOLS; ++k) {                                        \
        const int jj = wave + 4 * k; /* < VFP <= 64: a lane of the table */                    \
        const int ll = __builtin_amdgcn_readlane(cur.x, jj);                                   \
        const int b = __builtin_amdgcn_readlane(cur.y, jj);                                    \
        const int lo = ll & 0xffff, len = ll >> 16;                                            \
        stage_column<SP, PAIRED>(S, k, wb, qb, i, lo, (unsigned)len, (unsigned)b,              \
                                 (unsigned)(b + 2 * (lo + len) - 1), iw, iq);                  \
    }
    if (g.paired) {
        PGET_STAGE_COLUMNS(true)
    } else {
        PGET_STAGE_COLUMNS(false)
#pragma unroll
        for (int k = 0; k < VCOLS; ++k) {
            S.wm[k] = typename SP::w_t{};
            if constexpr (SP::DR) S.qm[k] = 0.0f;
        }
    }
#undef PGET_STAGE_COLUMNS
    if (has_next) S.ct = col_table(g, gcol, an, Wnx);
}

// Coefficients of f and mu that a staged point spreads: step*E*wt and
// kq*(T - R')*wt, plus those of the mirror angle's sample at the same point
// when the geometry is paired.  With a depth response the f coefficient sees
// the cotangent blended between the near and far planes by the sample's
// alpha, and the mu coefficient adds the far plane's term.  cv (and cvf):
// the point's column values.
template <typename SP>
__device__ __forceinline__ float2 stage_coef(const Stage<SP>& S, int k, float kq, float4 cv, float4 cvf)
{
    const float2 w = SP::w(S.w[k]), wm = SP::w(S.wm[k]);
    const float wt = cv.x, t = cv.y, wtm = cv.z, tm = cv.w;
    if constexpr (SP::DR) {
        const float wtf = cvf.x, tf = cvf.y, wtfm = cvf.z, tfm = cvf.w;
        const float ct = fmaf(S.al, wtf - wt, wt);
        const float ctm = fmaf(S.alm, wtfm - wtm, wtm);
        const float cf = fmaf(wm.x, ctm, w.x * ct);
        float sm = wt * (t - w.y);
        sm = fmaf(wtf, tf - S.q[k], sm);
        sm = fmaf(wtm, tm - wm.y, sm);
        sm = fmaf(wtfm, tfm - S.qm[k], sm);
        return make_float2(cf, kq * sm);
    } else {
        const float kw = kq * wt, kwm = kq * wtm;
        const float cf = fmaf(wm.x, wtm, w.x * wt);
        const float cm = fmaf(kwm, tm - wm.y, kw * (t - w.y));
        return make_float2(cf, cm);
    }
}

// Column values of a stage into the LDS column table (by the first wave).
template <typename SP>
__device__ __forceinline__ void stage_columns(float4* colv, float4* colvf, const Stage<SP>& S)
{
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64 && lane < VFP) {
        colv[lane] = S.cv;
        if constexpr (SP::DR) colvf[lane] = S.cvf;
    }
}

// Staged value of every lattice point of the window (stage_coef).
template <typename SP>
__device__ __forceinline__ void stage_store(float2* lat, const Stage<SP>& S, float kq, const float4* colv,
                                            const float4* colvf)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane >= VFP) return;
#pragma unroll
    for (int k = 0; k < VCOLS; ++k) {
        const int jj = wave + 4 * k;
        if (jj < VFP)
            lat[lane * LP + jj] = stage_coef(S, k, kq, colv[jj], SP::DR ? colvf[jj] : make_float4(0, 0, 0, 0));
    }
}

// Adds the staged coefficients of the rotated pair (a + n_angles/4 and its
// mirror, loaded over rot_window(W)) to the points of W they coincide with:
// point (row ii, column jj) of the rotated window is W's point (row
// W.wi - 1 - jj, column ii).  Every point has one owner thread.
template <typename SP>
__device__ __forceinline__ void stage_add_rot(float2* lat, const Stage<SP>& S, float kq, const Window& W,
                                              const float4* colv, const float4* colvf)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane >= W.wj) return;   // rows of the rotated window
#pragma unroll
    for (int k = 0; k < VCOLS; ++k) {
        const int jj = wave + 4 * k;
        if (jj < W.wi) {
            const float2 c = stage_coef(S, k, kq, colv[jj], SP::DR ? colvf[jj] : make_float4(0, 0, 0, 0));
            float2* p = lat + (W.wi - 1 - jj) * LP + lane;
            float2 v = *p;
            v.x += c.x;
            v.y += c.y;
            *p = v;
        }
    }
}

// tent(d) = max(0, 1 - |d|); med3 against [0, 1] lets the compiler fold it
// into the clamp bit of the subtraction
__device__ __forceinline__ float tent(float d)
{
    return __builtin_amdgcn_fmed3f(1.0f - fabsf(d), 0.0f, 1.0f);
}

template <typename SP, bool QUAD>
__global__ void __launch_bounds__(VJP_THREADS) __attribute__((amdgpu_waves_per_eu(SP::VJP_WAVES))) k_vjp_lin(VjpArgs A,
                                                                      const float4* __restrict__ trig,
                                                                      const int2* __restrict__ gcol)
{
    __shared__ float2 lat[VFP * LP];
    // column values of the staged windows (the angle's, the rotated pair's)
    __shared__ float4 colv[2][VFP];
    __shared__ float4 colvf[SP::DR ? 2 : 1][SP::DR ? VFP : 1];
    const Geo& g = A.g;
    // Workgroups go to the XCDs round-robin by linear id; give each XCD a
    // contiguous run of (slice, group, tile) items so that neighbouring tiles
    // (whose lattice windows overlap) share that XCD's L2.
    const int ntile = A.tiles_x * A.tiles_x;
    int item = xcd_item(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int tile = item % ntile;
    item /= ntile;
    const int grp = item % A.groups, slice = item / A.groups;
    if (A.st) {
        if (A.st[slice].done) return;
        if (A.skip_if_clean && !A.st[slice].dirty) return;
    }
    const int tr0 = (tile / A.tiles_x) * VT, tc0 = (tile % A.tiles_x) * VT;
    // a slot gathers angle a, its mirror (paired) and the quarter-turn pair
    // (QUAD).  The slots form A.fine groups of A.spf consecutive slots, each
    // summed into its own partial image (the plan fixes them, so a pixel's
    // additions run in the same order at every batch size); this block runs
    // the fine groups [grp * A.fpb, (grp + 1) * A.fpb).
    const int n_slots = QUAD ? g.n_angles / 4 : g.paired ? g.n_angles / 2 : g.n_angles;
    const int f_begin = grp * A.fpb, f_end = min(A.fine, f_begin + A.fpb);
    const int a_begin = f_begin * A.spf, a_end = min(n_slots, f_end * A.spf);
    const int qa = g.n_angles / 4;

    // this thread's 4 pixels: the same position in the four 8x8 blocks of its
    // wave's 16x16 quarter (a wave touches one compact 8x8 block per step)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int qr = tr0 + (wave >> 1) * 16, qc = tc0 + (wave & 1) * 16;
    // pixel b sits at (row0 + 8 (b >> 1), col0 + 8 (b & 1)); x, y centred
    const float x0 = (float)(qc + (lane & 7)) - g.half, y0 = (float)(qr + (lane >> 3)) - g.half;
    float accf[4] = {0.f, 0.f, 0.f, 0.f}, accm[4] = {0.f, 0.f, 0.f, 0.f};
    const float SQ2 = 1.41421356f;
    const float inv_ds = 1.0f / g.bin_size, inv_dt = 1.0f / g.step;
    const typename SP::w_t* wbase = static_cast<const typename SP::w_t*>(A.wts) + (size_t)slice * A.wts_stride;
    const float* qbase = SP::DR ? A.wq + (size_t)slice * A.wts_stride : nullptr;

    // End of fine group fg: its sum (this thread's 4 pixels, both maps) goes
    // either to its own partial image or, when the block runs whole super
    // groups, onto the running super-group sum kept in LDS (each thread its
    // own entries), written out at the super group's end.  Either way the
    // additions per pixel are: slots in order within a fine group, fine
    // groups in order within a super group, super groups in order (the last
    // two by the consumer for fine partials).
    __shared__ float2 tot[4 * VJP_THREADS];
    auto write_out = [&](int idx, const float* vf, const float* vm) {
        float* out = A.gpart + (size_t)idx * A.gpart_group_stride + (size_t)slice * A.gpart_slice_stride;
        const int n2 = g.n * g.n;
        // an empty asm on the thread index keeps the offset arithmetic here:
        // hoisted out of the loop it would hold registers across the gather
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int l = tid & 63, wv = tid >> 6;
        const int r0 = tr0 + (wv >> 1) * 16 + (l >> 3), c0 = tc0 + (wv & 1) * 16 + (l & 7);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int rr = r0 + (b >> 1) * 8, cc = c0 + (b & 1) * 8;
            if (rr < g.n && cc < g.n) {
                out[rr * g.n + cc] = vf[b];
                out[n2 + rr * g.n + cc] = vm[b];
            }
        }
    };
    if (A.super_out) {
#pragma unroll
        for (int b = 0; b < 4; ++b) tot[b * VJP_THREADS + threadIdx.x] = make_float2(0.0f, 0.0f);
    }
    auto flush = [&](int fg) {
        if (!A.super_out) {
            write_out(fg, accf, accm);
        } else {
            float tf[4], tm[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float2 t = tot[b * VJP_THREADS + threadIdx.x];
                t.x += accf[b];
                t.y += accm[b];
                tf[b] = t.x;
                tm[b] = t.y;
                tot[b * VJP_THREADS + threadIdx.x] = t;
            }
            if ((fg + 1) % A.gs == 0 || fg + 1 == A.fine) {
                write_out(fg / A.gs, tf, tm);
#pragma unroll
                for (int b = 0; b < 4; ++b) tot[b * VJP_THREADS + threadIdx.x] = make_float2(0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accf[b] = 0.0f;
            accm[b] = 0.0f;
        }
    };

    // `trig`, `clip` and `roff` are the plan's tables (A.t.*) as restrict
    // arguments: the compiler may then keep their loads scalar despite the
    // partial-image stores inside the loop (a vector load here would wait
    // for the next angle's weight loads in flight).
    // Wn: the window of the next angle to gather, Wnn: of the one after
    // (whose column table is read one angle ahead).
    Stage<SP> S, R;
    Window Wn = {0, 0, 0, 0}, Wnn = Wn;
    if (a_begin < a_end) {
        Wn = tile_window(g, trig[a_begin], tr0, tc0);
        const bool nx = a_begin + 1 < a_end;
        Wnn = nx ? tile_window(g, trig[a_begin + 1], tr0, tc0) : Wn;
        S.ct = col_table(g, gcol, a_begin, Wn);
        if (QUAD) R.ct = col_table(g, gcol, a_begin + qa, rot_window(g, Wn));
        stage_load<SP>(S, A, wbase, qbase, slice, a_begin, Wn, nx, a_begin + 1, Wnn, gcol);
        if (QUAD)
            stage_load<SP>(R, A, wbase, qbase, slice, a_begin + qa, rot_window(g, Wn), nx, a_begin + 1 + qa,
                           rot_window(g, Wnn), gcol);
    }
    int fg = f_begin, left = A.spf;   // fine group being summed, its slots still to come
    for (int a = a_begin; a < a_end; ++a) {
        const Window W = Wn;
        // no wave reads the column tables after the previous iteration's
        // staging barriers
        stage_columns(colv[0], colvf[0], S);
        if (QUAD) stage_columns(colv[1], colvf[SP::DR ? 1 : 0], R);
        __syncthreads();   // the previous angle's gather is done with lat; columns visible
        stage_store(lat, S, g.kq, colv[0], colvf[0]);
        if (QUAD) {
            __syncthreads();
            stage_add_rot(lat, R, g.kq, W, colv[1], colvf[SP::DR ? 1 : 0]);
        }
        __syncthreads();
        // the previous fine group is complete: write it out here, where the
        // staged registers are consumed and the next ones not yet loaded
        if (left == 0) {
            flush(fg++);
            left = A.spf;
        }
        if (a + 1 < a_end) {   // next angle's loads fly during this gather
            Wn = Wnn;
            const bool nx = a + 2 < a_end;
            if (nx) Wnn = tile_window(g, trig[a + 2], tr0, tc0);
            stage_load<SP>(S, A, wbase, qbase, slice, a + 1, Wn, nx, a + 2, Wnn, gcol);
            if (QUAD)
                stage_load<SP>(R, A, wbase, qbase, slice, a + 1 + qa, rot_window(g, Wn), nx, a + 2 + qa,
                               rot_window(g, Wnn), gcol);
        }
        const float4 tr = trig[a];
        const float cs = tr.z, sn = tr.w;
        // displacement (pixel -> lattice point) per unit lattice step, and its
        // value at the 3x3 candidate offsets (built from sums: no 0*x or 2*x)
        const float A1 = -g.bin_size * sn, A2 = g.step * cs;   // dx
        const float A3 = g.bin_size * cs, A4 = g.step * sn;    // dy
        const float oxj[3] = {0.0f, A1, A1 + A1}, oxi[3] = {0.0f, A2, A2 + A2};
        const float oyj[3] = {0.0f, A3, A3 + A3}, oyi[3] = {0.0f, A4, A4 + A4};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float x = x0 + (float)((b & 1) * 8), y = y0 + (float)((b >> 1) * 8);
            const float u = fmaf(-x * sn + y * cs, inv_ds, g.s_off);
            const float v = fmaf(x * cs + y * sn, inv_dt, g.t_off);
            const float ju = floorf(u - SQ2) + 1.0f, iv = floorf(v - SQ2) + 1.0f;
            const float du0 = ju - u, dv0 = iv - v;
            const float dx0 = fmaf(du0, A1, dv0 * A2), dy0 = fmaf(du0, A3, dv0 * A4);
            const int jb = min(max((int)ju - W.jlo, 0), VFP - 3);
            const int ib = min(max((int)iv - W.ilo, 0), VFP - 3);
            const float2* L = lat + ib * LP + jb;
            float sf = 0.0f, sm = 0.0f;
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const float rx = dx0 + oxi[di], ry = dy0 + oyi[di];
#pragma unroll
                for (int dj = 0; dj < 3; ++dj) {
                    const float w = tent(rx + oxj[dj]) * tent(ry + oyj[dj]);
                    const float2 c = L[di * LP + dj];
                    sf = fmaf(w, c.x, sf);
                    sm = fmaf(w, c.y, sm);
                }
            }
            accf[b] += sf;
            accm[b] += sm;
        }
        --left;
    }
    flush(fg);
}

// Zero fill (kernels, not memset, so that captured graphs stay clean).
__global__ void __launch_bounds__(256) k_fill_zero(float4* p, long long n4)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Sum of the gather's partial images at element m of a slice (f block at
// m, mu block at n2 + m): runs of gfold partials (the fine groups of one
// super group; 1 when the partials are super-group sums) are added in
// order, then the runs in order -- the order the gather itself uses when it
// sums whole super groups, so both layouts give the same bits.  The loads
// of eight partials are issued before their adds so that they overlap.
__device__ __forceinline__ float2 sum_groups(const float* gp, long long group_stride, int groups, int gfold,
                                             int m, int n2)
{
    float sf = 0.0f, sm = 0.0f, tf = 0.0f, tm = 0.0f;
    int in_run = 0;
    auto add = [&](float vf, float vm) {
        tf += vf;
        tm += vm;
        if (++in_run == gfold) {
            sf += tf;
            sm += tm;
            tf = 0.0f;
            tm = 0.0f;
            in_run = 0;
        }
    };
    int k = 0;
    for (; k + 8 <= groups; k += 8) {
        float vf[8], vm[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            vf[u] = gp[(size_t)(k + u) * group_stride + m];
            vm[u] = gp[(size_t)(k + u) * group_stride + n2 + m];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) add(vf[u], vm[u]);
    }
    for (; k < groups; ++k) add(gp[(size_t)k * group_stride + m], gp[(size_t)k * group_stride + n2 + m]);
    if (in_run > 0) {
        sf += tf;
        sm += tm;
    }
    return make_float2(sf, sm);
}

// Sum of the gather's partial images (fixed order) into gf / gm.
__global__ void __launch_bounds__(256) k_sum_groups(int n2, int groups, int gfold, const float* gpart,
                                                    long long group_stride, float* gf, float* gm)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n2) return;
    const float2 s = sum_groups(gpart, group_stride, groups, gfold, idx, n2);
    gf[idx] = s.x;
    gm[idx] = s.y;
}

// ----------------------------------------------------------- LM kernels
// Vectors of one slice are [2][N][N] (f block, then mu block).

// Scaled gradient projection (Bonettini, Zanella and Zanni): Armijo
// sufficient decrease and backtracking ratio, steplength bounds, the first
// steplength and the first alternation threshold.
constexpr double SGP_ARMIJO = 1e-4;
constexpr double SGP_BACKTRACK = 0.4;
constexpr double SGP_ALPHA_MIN = 1e-10;
constexpr double SGP_ALPHA_MAX = 1e5;
constexpr float SGP_ALPHA0 = 1.0f;
constexpr double SGP_TAU0 = 0.5;

__device__ __forceinline__ void alphas_at(const LMParamsDev& p, int k, float& af, float& am)
{
    int e = min(k, p.alpha_decay_until);
    double d = pow(p.alpha_decay, (double)e);
    af = (float)(p.alpha_f / d);
    am = (float)(p.alpha_mu / d);
}

// Continuation factor of the geometry prior's weights at outer iteration k
// (the same division as the alphas').
__device__ __forceinline__ float prior_scale(const LMParamsDev& p, int k)
{
    int e = min(k, p.alpha_decay_until);
    return (float)(1.0 / pow(p.alpha_decay, (double)e));
}

// Weight and reference of the geometry prior for element mm of a slice's
// (f, mu) pair (0 <= mm < 2 N^2), scaled by ps; zero weight without a prior.
__device__ __forceinline__ void prior_at(const LMParamsDev& p, float ps, int mm, float& w, float& ref)
{
    w = p.prior_w ? ps * p.prior_w[mm] : 0.0f;
    ref = p.prior_ref ? p.prior_ref[mm] : 0.0f;
}

// L x at pixel (r, c): sum over in-grid 4-neighbours of (x[m] - x[m'])
__device__ __forceinline__ float lap(const float* x, int n, int r, int c)
{
    const int m = r * n + c;
    const float v = x[m];
    float acc = 0.0f;
    if (c > 0) acc += v - x[m - 1];
    if (c + 1 < n) acc += v - x[m + 1];
    if (r > 0) acc += v - x[m - n];
    if (r + 1 < n) acc += v - x[m + n];
    return acc;
}

// squared forward differences at pixel (r, c) (right and down edges)
__device__ __forceinline__ float grad2(const float* x, int n, int r, int c)
{
    const int m = r * n + c;
    float acc = 0.0f;
    if (c + 1 < n) { float d = x[m + 1] - x[m]; acc += d * d; }
    if (r + 1 < n) { float d = x[m + n] - x[m]; acc += d * d; }
    return acc;
}

// Start of an outer iteration: g = J^T (A(u) - y) + R u;  CG state x = 0,
// r = -F g (F: the free-variable mask when the active set is on, else 1),
// p = 0;  partials of r.W r, ||g||^2 and alpha ||grad u||^2.
__global__ void __launch_bounds__(EW_THREADS) k_grad_init(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    LMState& st = V.st[slice];
    if (st.done) return;
    const Geo& g = V.g;
    const int n = g.n, n2 = n * n;
    float af, am;
    alphas_at(V.prm[slice], st.k, af, am);
    const size_t vo = (size_t)slice * V.vstride;
    const float* gp = V.gpart + (size_t)slice * V.gpart_slice_stride;
    const LMParamsDev& P = V.prm[slice];
    double rr = 0.0, gg = 0.0, reg = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        const int r = m / n, c = m - r * n;
        const float* uf = V.u + vo;
        const float* um = uf + n2;
        const float2 gs = sum_groups(gp, V.gpart_group_stride, V.groups, V.gfold, m, n2);
        float gf = gs.x, gm = gs.y;
        gf = fmaf(af, lap(uf, n, r, c), gf);
        gm = fmaf(am, lap(um, n, r, c), gm);
        double prior_e = 0.0;
        if (P.prior_w) {
            const float ps = prior_scale(P, st.k);
            float wf, rf0, wm, rm0;
            prior_at(P, ps, m, wf, rf0);
            prior_at(P, ps, n2 + m, wm, rm0);
            const float df = uf[m] - rf0, dm = um[m] - rm0;
            gf = fmaf(wf, df, gf);
            gm = fmaf(wm, dm, gm);
            prior_e = (double)wf * ((double)df * df) + (double)wm * ((double)dm * dm);
        }
        V.grad[vo + m] = gf;
        V.grad[vo + n2 + m] = gm;
        const float f0 = uf[m], m0 = um[m];
        if (P.step_sgp) {
            // scaled gradient projection from s = 0: r = grad q(0) = g and the
            // first direction d = P_box(-alpha_0 W g) in step space
            V.r[vo + m] = gf;
            V.r[vo + n2 + m] = gm;
            V.p[vo + m] = fminf(fmaxf(-SGP_ALPHA0 * (float)P.w_f * gf, (float)P.f_lo - f0), (float)P.f_hi - f0);
            V.p[vo + n2 + m] = fminf(fmaxf(-SGP_ALPHA0 * (float)P.w_mu * gm, (float)P.mu_lo - m0), (float)P.mu_hi - m0);
            V.fmask[vo + m] = 1;
            V.fmask[vo + n2 + m] = 1;
        } else {
            float rf = -gf, rm = -gm;
            if (P.active_set) {
                // held: on the lower bound with g > 0, or on the upper bound with g < 0
                const bool hold_f = (f0 <= (float)P.f_lo && gf > 0.0f) || (f0 >= (float)P.f_hi && gf < 0.0f);
                const bool hold_m = (m0 <= (float)P.mu_lo && gm > 0.0f) || (m0 >= (float)P.mu_hi && gm < 0.0f);
                V.fmask[vo + m] = hold_f ? 0 : 1;
                V.fmask[vo + n2 + m] = hold_m ? 0 : 1;
                if (hold_f) rf = 0.0f;
                if (hold_m) rm = 0.0f;
            }
            V.r[vo + m] = rf;
            V.r[vo + n2 + m] = rm;
            V.p[vo + m] = 0.0f;
            V.p[vo + n2 + m] = 0.0f;
            rr = (double)(float)P.w_f * ((double)rf * rf) + (double)(float)P.w_mu * ((double)rm * rm);
        }
        V.x[vo + m] = 0.0f;
        V.x[vo + n2 + m] = 0.0f;
        gg = (double)gf * gf + (double)gm * gm;
        reg = (double)af * grad2(uf, n, r, c) + (double)am * grad2(um, n, r, c) + prior_e;
    }
    if (P.step_sgp && blockIdx.x == 0 && threadIdx.x == 0) {
        st.sgp_alpha = SGP_ALPHA0;
        st.sgp_tau = SGP_TAU0;
        st.sgp_nbb = 0;
        st.sgp_q = 0.0;
        st.sgp_lambda = 0.0;
    }
    double s1 = block_sum(rr, sh);
    double s3 = block_sum(gg, sh);
    double s2 = block_sum(reg, sh);
    if (threadIdx.x == 0) {
        slot_ptr(V.part, slice, SLOT_RR0)[blockIdx.x] = s1;
        slot_ptr(V.part, slice, SLOT_GNORM)[blockIdx.x] = s3;
        slot_ptr(V.part, slice, SLOT_PHI_REG_U)[blockIdx.x] = s2;
    }
}

// CG step, first half: p = W r + beta_cg p_old (beta_cg = rr_m / rr_{m-1},
// rr = r.W r), q = F (J^T J p + beta D p + R p), partials of gamma = p.q.
__global__ void __launch_bounds__(EW_THREADS) k_cg_q(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    LMState& st = V.st[slice];
    if (st.done) return;
    const Geo& g = V.g;
    const int n = g.n, n2 = n * n;
    const int m_step = V.cg_step;
    float bcg = 0.0f;
    double rr_cur = sum_partials(slot_ptr(V.part, slice, rr_slot(m_step)), V.n_ew_blocks, sh);
    if (m_step > 0) {
        double rr_prev = sum_partials(slot_ptr(V.part, slice, rr_slot(m_step + 2)), V.n_ew_blocks, sh);
        bcg = rr_prev > 0.0 ? (float)(rr_cur / rr_prev) : 0.0f;
        if (blockIdx.x == 0 && threadIdx.x == 0 && V.rep)
            V.rep[slice].cg_rr[(size_t)st.k * V.prm[slice].n_cg + (m_step - 1)] = rr_cur;
    } else if (blockIdx.x == 0 && V.rep) {
        const double gg = sum_partials(slot_ptr(V.part, slice, SLOT_GNORM), V.n_ew_blocks, sh);
        if (threadIdx.x == 0) V.rep[slice].gnorm[st.k] = sqrt(gg);
    }
    float af, am;
    alphas_at(V.prm[slice], st.k, af, am);
    const float bdf = (float)(st.beta * V.prm[slice].d_f), bdm = (float)(st.beta * V.prm[slice].d_mu);
    const float wf = (float)V.prm[slice].w_f, wm = (float)V.prm[slice].w_mu;
    const int act = V.prm[slice].active_set;
    const size_t vo = (size_t)slice * V.vstride;
    const float* gp = V.gpart + (size_t)slice * V.gpart_slice_stride;
    double gam = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        const int r = m / n, c = m - r * n;
        const float* rf = V.r + vo;
        const float* rm = rf + n2;
        const float* pf = V.p + vo;
        const float* pm = pf + n2;
        // p at the pixel and its 4 neighbours
        auto PF = [&](int mm) { return fmaf(bcg, pf[mm], wf * rf[mm]); };
        auto PM = [&](int mm) { return fmaf(bcg, pm[mm], wm * rm[mm]); };
        const float pfc = PF(m), pmc = PM(m);
        float lf = 0.0f, lm = 0.0f;
        if (c > 0) { lf += pfc - PF(m - 1); lm += pmc - PM(m - 1); }
        if (c + 1 < n) { lf += pfc - PF(m + 1); lm += pmc - PM(m + 1); }
        if (r > 0) { lf += pfc - PF(m - n); lm += pmc - PM(m - n); }
        if (r + 1 < n) { lf += pfc - PF(m + n); lm += pmc - PM(m + n); }
        const float2 gs = sum_groups(gp, V.gpart_group_stride, V.groups, V.gfold, m, n2);
        const float gf = gs.x, gm = gs.y;
        float qf = fmaf(af, lf, fmaf(bdf, pfc, gf));
        float qm = fmaf(am, lm, fmaf(bdm, pmc, gm));
        if (V.prm[slice].prior_w) {
            const float ps = prior_scale(V.prm[slice], st.k);
            float wf, wm, rf0, rm0;
            prior_at(V.prm[slice], ps, m, wf, rf0);
            prior_at(V.prm[slice], ps, n2 + m, wm, rm0);
            qf = fmaf(wf, pfc, qf);
            qm = fmaf(wm, pmc, qm);
        }
        if (act) {
            if (!V.fmask[vo + m]) qf = 0.0f;
            if (!V.fmask[vo + n2 + m]) qm = 0.0f;
        }
        V.q[vo + m] = qf;
        V.q[vo + n2 + m] = qm;
        gam = (double)pfc * qf + (double)pmc * qm;
    }
    double s = block_sum(gam, sh);
    if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_GAMMA)[blockIdx.x] = s;
}

// CG step, second half: alpha = rr_m / gamma; x += alpha p; r -= alpha q;
// p_old <- p; partials of rr_{m+1} = r.W r.
__global__ void __launch_bounds__(EW_THREADS) k_cg_x(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    LMState& st = V.st[slice];
    if (st.done) return;
    const Geo& g = V.g;
    const int n2 = g.n * g.n;
    const int m_step = V.cg_step;
    double rr_cur = sum_partials(slot_ptr(V.part, slice, rr_slot(m_step)), V.n_ew_blocks, sh);
    float bcg = 0.0f;
    if (m_step > 0) {
        double rr_prev = sum_partials(slot_ptr(V.part, slice, rr_slot(m_step + 2)), V.n_ew_blocks, sh);
        bcg = rr_prev > 0.0 ? (float)(rr_cur / rr_prev) : 0.0f;
    }
    double gam = sum_partials(slot_ptr(V.part, slice, SLOT_GAMMA), V.n_ew_blocks, sh);
    const float alpha = (gam > 0.0 && rr_cur > 0.0) ? (float)(rr_cur / gam) : 0.0f;
    const size_t vo = (size_t)slice * V.vstride;
    const float w2[2] = {(float)V.prm[slice].w_f, (float)V.prm[slice].w_mu};
    double rr = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const size_t o = vo + (size_t)b * n2 + m;
            const float p = fmaf(bcg, V.p[o], w2[b] * V.r[o]);
            V.x[o] = fmaf(alpha, p, V.x[o]);
            const float rn = fmaf(-alpha, V.q[o], V.r[o]);
            V.r[o] = rn;
            V.p[o] = p;
            rr += (double)w2[b] * ((double)rn * rn);
        }
    }
    double s = block_sum(rr, sh);
    if (threadIdx.x == 0) slot_ptr(V.part, slice, rr_slot(m_step + 1))[blockIdx.x] = s;
}

// ---- scaled gradient projection of the box-constrained step (Sec. 2.2,
// after Bonettini, Zanella and Zanni): x holds the step s, r the gradient
// grad q(s) = g + M s, p the direction d, q the product M d.

// M d = (J^T J + beta D + R) d from the gather's partials, and the partials
// of grad q . d, d.M d and the four scaled Barzilai-Borwein sums.
__global__ void __launch_bounds__(EW_THREADS) k_sgp_q(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    LMState& st = V.st[slice];
    if (st.done) return;
    const Geo& g = V.g;
    const int n = g.n, n2 = n * n;
    const LMParamsDev& P = V.prm[slice];
    float af, am;
    alphas_at(P, st.k, af, am);
    const float bdf = (float)(st.beta * P.d_f), bdm = (float)(st.beta * P.d_mu);
    const float wf = (float)P.w_f, wm = (float)P.w_mu;
    const size_t vo = (size_t)slice * V.vstride;
    const float* gp = V.gpart + (size_t)slice * V.gpart_slice_stride;
    double gd = 0.0, dmd = 0.0, n1 = 0.0, d1 = 0.0, nn2 = 0.0, d2 = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        const int r = m / n, c = m - r * n;
        const float* pf = V.p + vo;
        const float* pm = pf + n2;
        const float2 gs = sum_groups(gp, V.gpart_group_stride, V.groups, V.gfold, m, n2);
        float qf = fmaf(af, lap(pf, n, r, c), fmaf(bdf, pf[m], gs.x));
        float qm = fmaf(am, lap(pm, n, r, c), fmaf(bdm, pm[m], gs.y));
        if (P.prior_w) {
            const float ps = prior_scale(P, st.k);
            float pwf, pwm, rf0, rm0;
            prior_at(P, ps, m, pwf, rf0);
            prior_at(P, ps, n2 + m, pwm, rm0);
            qf = fmaf(pwf, pf[m], qf);
            qm = fmaf(pwm, pm[m], qm);
        }
        V.q[vo + m] = qf;
        V.q[vo + n2 + m] = qm;
        const double df = pf[m], dm = pm[m], Qf = qf, Qm = qm;
        const double Wf = wf, Wm = wm;
        gd = (double)V.r[vo + m] * df + (double)V.r[vo + n2 + m] * dm;
        dmd = df * Qf + dm * Qm;
        n1 = df * df / (Wf * Wf) + dm * dm / (Wm * Wm);
        d1 = df * Qf / Wf + dm * Qm / Wm;
        nn2 = Wf * df * Qf + Wm * dm * Qm;
        d2 = Wf * Wf * Qf * Qf + Wm * Wm * Qm * Qm;
    }
    double v;
    v = block_sum(gd, sh);  if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_GD)[blockIdx.x] = v;
    v = block_sum(dmd, sh); if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_DMD)[blockIdx.x] = v;
    v = block_sum(n1, sh);  if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_N1)[blockIdx.x] = v;
    v = block_sum(d1, sh);  if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_D1)[blockIdx.x] = v;
    v = block_sum(nn2, sh); if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_N2)[blockIdx.x] = v;
    v = block_sum(d2, sh);  if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SGP_D2)[blockIdx.x] = v;
}

// Per slice: the Armijo factor lambda (1, 0.4, 0.16, ... until
// q(s + lambda d) <= q(s) + 1e-4 lambda grad q . d, exact for the quadratic),
// q(s) after the move, and the next steplength from the scaled
// Barzilai-Borwein rules with alternation.  No descent (grad q . d >= 0):
// lambda = 0 and the steplength is kept.
__global__ void __launch_bounds__(256) k_sgp_step(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.x;
    LMState& st = V.st[slice];
    if (st.done) return;
    const LMParamsDev& P = V.prm[slice];
    const double gd = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_GD), V.n_ew_blocks, sh);
    const double dmd = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_DMD), V.n_ew_blocks, sh);
    const double n1 = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_N1), V.n_ew_blocks, sh);
    const double d1 = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_D1), V.n_ew_blocks, sh);
    const double n2 = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_N2), V.n_ew_blocks, sh);
    const double d2 = sum_partials(slot_ptr(V.part, slice, SLOT_SGP_D2), V.n_ew_blocks, sh);
    double gg = 0.0;
    if (V.cg_step == 0 && V.rep) gg = sum_partials(slot_ptr(V.part, slice, SLOT_GNORM), V.n_ew_blocks, sh);
    if (threadIdx.x != 0) return;
    if (V.cg_step == 0 && V.rep) V.rep[slice].gnorm[st.k] = sqrt(gg);
    double lam = 0.0;
    if (gd < 0.0) {
        lam = 1.0;
        while (lam * gd + 0.5 * lam * lam * dmd > SGP_ARMIJO * lam * gd && lam > 1e-30) lam *= SGP_BACKTRACK;
        st.sgp_q += lam * gd + 0.5 * lam * lam * dmd;
        const double bb1 = d1 > 0.0 ? n1 / d1 : SGP_ALPHA_MAX;
        const double bb2 = n2 > 0.0 ? n2 / d2 : SGP_ALPHA_MAX;
        if (st.sgp_nbb < 3) {
            st.sgp_bb2[st.sgp_nbb++] = bb2;
        } else {
            st.sgp_bb2[0] = st.sgp_bb2[1];
            st.sgp_bb2[1] = st.sgp_bb2[2];
            st.sgp_bb2[2] = bb2;
        }
        double alpha;
        if (bb2 / bb1 <= st.sgp_tau) {
            alpha = st.sgp_bb2[0];
            for (int i = 1; i < st.sgp_nbb; ++i) alpha = fmin(alpha, st.sgp_bb2[i]);
            st.sgp_tau *= 0.9;
        } else {
            alpha = bb1;
            st.sgp_tau *= 1.1;
        }
        st.sgp_alpha = fmin(fmax(alpha, SGP_ALPHA_MIN), SGP_ALPHA_MAX);
    }
    st.sgp_lambda = lam;
    if (V.rep) V.rep[slice].cg_rr[(size_t)st.k * P.n_cg + V.cg_step] = st.sgp_q;
}

// s += lambda d, grad q += lambda M d, and the next direction
// d = P_box(s - alpha W grad q) - s with the new steplength.
__global__ void __launch_bounds__(EW_THREADS) k_sgp_x(VecArgs V)
{
    const int slice = blockIdx.y;
    const LMState& st = V.st[slice];
    if (st.done) return;
    const LMParamsDev& P = V.prm[slice];
    const int n2 = V.g.n * V.g.n;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n2) return;
    const float lam = (float)st.sgp_lambda, alpha = (float)st.sgp_alpha;
    const size_t vo = (size_t)slice * V.vstride;
    const float w2[2] = {(float)P.w_f, (float)P.w_mu};
    const float lo2[2] = {(float)P.f_lo, (float)P.mu_lo}, hi2[2] = {(float)P.f_hi, (float)P.mu_hi};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const size_t o = vo + (size_t)b * n2 + m;
        const float x = fmaf(lam, V.p[o], V.x[o]);
        const float r = fmaf(lam, V.q[o], V.r[o]);
        const float u = V.u[o];
        V.x[o] = x;
        V.r[o] = r;
        V.p[o] = fminf(fmaxf(fmaf(-alpha * w2[b], r, x), lo2[b] - u), hi2[b] - u) - x;
    }
}

// Trial point u' = clamp(u + x) (or the hook's proposal), s = u' - u, and
// partials of g.s, s.R s, ||s||^2, ||u||^2, alpha ||grad u'||^2.
__global__ void __launch_bounds__(EW_THREADS) k_trial(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    LMState& st = V.st[slice];
    if (st.done) return;
    const LMParamsDev& P = V.prm[slice];
    const Geo& g = V.g;
    const int n = g.n, n2 = n * n;
    if (!V.hook_mode && V.rep && blockIdx.x == 0 && !P.step_sgp) {
        double rr = sum_partials(slot_ptr(V.part, slice, rr_slot(P.n_cg)), V.n_ew_blocks, sh);
        if (threadIdx.x == 0) V.rep[slice].cg_rr[(size_t)st.k * P.n_cg + (P.n_cg - 1)] = rr;
    }
    float af, am;
    alphas_at(P, st.k, af, am);
    const size_t vo = (size_t)slice * V.vstride;
    const float* uf = V.u + vo;
    const float* um = uf + n2;
    const float lo_f = (float)P.f_lo, hi_f = (float)P.f_hi, lo_m = (float)P.mu_lo, hi_m = (float)P.mu_hi;
    auto TF = [&](int mm) {
        return V.hook_mode ? V.ut[vo + mm] : fminf(fmaxf(uf[mm] + V.x[vo + mm], lo_f), hi_f);
    };
    auto TM = [&](int mm) {
        return V.hook_mode ? V.ut[vo + n2 + mm] : fminf(fmaxf(um[mm] + V.x[vo + n2 + mm], lo_m), hi_m);
    };
    double gs = 0.0, srs = 0.0, ss = 0.0, uu = 0.0, regt = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        const int r = m / n, c = m - r * n;
        const float tf = TF(m), tm = TM(m);
        const float sf = tf - uf[m], sm = tm - um[m];
        float gsf = 0.0f, gsm = 0.0f, gtf = 0.0f, gtm = 0.0f;
        if (c + 1 < n) {
            const float tf1 = TF(m + 1), tm1 = TM(m + 1);
            const float df = (tf1 - uf[m + 1]) - sf, dm = (tm1 - um[m + 1]) - sm;
            gsf += df * df; gsm += dm * dm;
            const float ef = tf1 - tf, em = tm1 - tm;
            gtf += ef * ef; gtm += em * em;
        }
        if (r + 1 < n) {
            const float tf1 = TF(m + n), tm1 = TM(m + n);
            const float df = (tf1 - uf[m + n]) - sf, dm = (tm1 - um[m + n]) - sm;
            gsf += df * df; gsm += dm * dm;
            const float ef = tf1 - tf, em = tm1 - tm;
            gtf += ef * ef; gtm += em * em;
        }
        if (!V.hook_mode) {
            V.ut[vo + m] = tf;
            V.ut[vo + n2 + m] = tm;
        }
        V.s[vo + m] = sf;
        V.s[vo + n2 + m] = sm;
        gs = (double)V.grad[vo + m] * sf + (double)V.grad[vo + n2 + m] * sm;
        srs = (double)af * gsf + (double)am * gsm;
        ss = (double)sf * sf + (double)sm * sm;
        uu = (double)uf[m] * uf[m] + (double)um[m] * um[m];
        regt = (double)af * gtf + (double)am * gtm;
        if (P.prior_w) {
            const float ps = prior_scale(P, st.k);
            float wf, wm, rf0, rm0;
            prior_at(P, ps, m, wf, rf0);
            prior_at(P, ps, n2 + m, wm, rm0);
            const float ef = tf - rf0, em = tm - rm0;
            srs += (double)wf * ((double)sf * sf) + (double)wm * ((double)sm * sm);
            regt += (double)wf * ((double)ef * ef) + (double)wm * ((double)em * em);
        }
    }
    double v;
    v = block_sum(gs, sh);   if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_GS)[blockIdx.x] = v;
    v = block_sum(srs, sh);  if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SRS)[blockIdx.x] = v;
    v = block_sum(ss, sh);   if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_SNORM)[blockIdx.x] = v;
    v = block_sum(uu, sh);   if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_UNORM)[blockIdx.x] = v;
    v = block_sum(regt, sh); if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_PHI_REG_T)[blockIdx.x] = v;
}

// Iterate trace (optional, per slice): u_k and the trial point u'_k of the
// current outer iteration into rows k of the caller's buffers.
__global__ void __launch_bounds__(EW_THREADS) k_trace(VecArgs V)
{
    const int slice = blockIdx.y;
    const LMState& st = V.st[slice];
    const LMParamsDev& P = V.prm[slice];
    if (st.done || (!P.trace_u && !P.trace_t)) return;
    const long long n2x2 = V.vstride;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= V.g.n * V.g.n) return;
    const size_t vo = (size_t)slice * n2x2;
    const size_t row = (size_t)st.k * n2x2;
    const int n2 = V.g.n * V.g.n;
    if (P.trace_u) {
        P.trace_u[row + m] = V.u[vo + m];
        P.trace_u[row + n2 + m] = V.u[vo + n2 + m];
    }
    if (P.trace_t) {
        P.trace_t[row + m] = V.ut[vo + m];
        P.trace_t[row + n2 + m] = V.ut[vo + n2 + m];
    }
}

// Initial damping: beta0 = tau ||J 1||^2 / (2 N^2) unless given.
__global__ void __launch_bounds__(256) k_beta0(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.x;
    LMState& st = V.st[slice];
    const LMParamsDev& P = V.prm[slice];
    if (st.done || st.k != 0) return;   // block-uniform
    double j1 = sum_partials(slot_ptr(V.part, slice, SLOT_J1), V.n_angle_parts, sh);
    if (threadIdx.x == 0 && P.beta0 <= 0.0) {
        const double n2 = (double)V.g.n * V.g.n;
        st.beta = P.tau * j1 / (2.0 * n2);
        st.beta_init = st.beta;
        if (!(st.beta > 0.0) || !isfinite(st.beta)) {
            st.status = -4;
            st.stop_reason = 3;
            st.done = 1;
        }
    }
}

// Per-slice solver state at the start of a solve: beta from the parameters
// (or left for k_beta0), nu = 2, k = 0, the iterate marked for linearising.
__global__ void k_lm_init(LMState* st, const LMParamsDev* prm, int n_slices)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    LMState z = {};
    z.beta = prm[s].beta0 > 0.0 ? prm[s].beta0 : 0.0;
    z.beta_init = z.beta;
    z.nu = 2.0;
    z.dirty = 1;
    z.final_slot = SLOT_PHI_DATA_U;
    st[s] = z;
}

// Gain ratio test and damping update (one block per slice).
__global__ void __launch_bounds__(256) k_decide(VecArgs V, int hook_present)
{
    __shared__ double sh[16];
    const int slice = blockIdx.x;
    LMState& st = V.st[slice];
    if (st.done) return;
    const LMParamsDev& P = V.prm[slice];
    const double phid_u = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_DATA_U), V.n_angle_parts, sh);
    const double regu = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_REG_U), V.n_ew_blocks, sh);
    const double phid_t = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_DATA_T), V.n_angle_parts, sh);
    const double regt = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_REG_T), V.n_ew_blocks, sh);
    const double gs = sum_partials(slot_ptr(V.part, slice, SLOT_GS), V.n_ew_blocks, sh);
    const double srs = sum_partials(slot_ptr(V.part, slice, SLOT_SRS), V.n_ew_blocks, sh);
    const double js = sum_partials(slot_ptr(V.part, slice, SLOT_JS), V.n_angle_parts, sh);
    const double ss = sum_partials(slot_ptr(V.part, slice, SLOT_SNORM), V.n_ew_blocks, sh);
    const double uu = sum_partials(slot_ptr(V.part, slice, SLOT_UNORM), V.n_ew_blocks, sh);
    if (threadIdx.x != 0) return;
    (void)hook_present;
    const int k = st.k;
    const double phi_u = 0.5 * phid_u + 0.5 * regu;
    const double phi_t = 0.5 * phid_t + 0.5 * regt;
    const double pred = -(gs + 0.5 * (js + srs));
    const double ared = phi_u - phi_t;
    const double rho = pred > 0.0 ? ared / pred : -INFINITY;
    const int acc = P.has_replay ? (P.replay[k] != 0) : (rho > P.eta);
    if (V.rep) {
        ReportDev& R = V.rep[slice];
        R.phi[k] = phi_u;
        R.rho[k] = rho;
        R.beta[k] = st.beta;
        R.pred[k] = pred;
        R.ared[k] = ared;
        R.accepted[k] = (int8_t)acc;
        R.hook_accepted[k] = 0;
        R.hook_rho[k] = NAN;
        R.hook_pred[k] = NAN;
    }
    st.phi_u = phi_u;
    st.pred = pred;
    st.ared = ared;
    st.rho = rho;
    st.hook_keep = 0;
    st.k = k + 1;
    if (!isfinite(phi_u)) {
        st.status = -4;
        st.stop_reason = 3;
        st.accepted = 0;
        st.done_next = 1;
        return;
    }
    if (acc) {
        const double t = 2.0 * rho - 1.0;
        const double fct = 1.0 - t * t * t;
        st.beta *= (fct > 1.0 / 3.0 ? fct : 1.0 / 3.0);
        st.nu = 2.0;
        st.final_slot = SLOT_PHI_DATA_T;
    } else {
        st.beta *= st.nu;
        st.nu *= 2.0;
        st.final_slot = SLOT_PHI_DATA_U;
    }
    st.accepted = acc;
    st.dirty = acc;
    if (acc && P.tol > 0.0 && (ared <= P.tol * phi_u || sqrt(ss) <= P.tol * sqrt(uu))) {
        st.stop_reason = 1;
        st.done_next = 1;
    }
    if (!(st.beta <= 1e16 * st.beta_init)) {
        st.stop_reason = 2;
        st.done_next = 1;
    }
}

// Safeguard of a hook proposal u~ (Prop. 3.2, Alg. 2): keep it iff
// rho(s~) > eta and m(s~) <= m(s), i.e. pred(s~) >= pred(s).
__global__ void __launch_bounds__(256) k_hook_decide(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.x;
    LMState& st = V.st[slice];
    if (st.done || !st.accepted) return;
    const LMParamsDev& P = V.prm[slice];
    const double phid_h = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_DATA_H), V.n_angle_parts, sh);
    const double regt = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_REG_T), V.n_ew_blocks, sh);
    const double gs = sum_partials(slot_ptr(V.part, slice, SLOT_GS), V.n_ew_blocks, sh);
    const double srs = sum_partials(slot_ptr(V.part, slice, SLOT_SRS), V.n_ew_blocks, sh);
    const double js = sum_partials(slot_ptr(V.part, slice, SLOT_JS), V.n_angle_parts, sh);
    if (threadIdx.x != 0) return;
    const double phi_h = 0.5 * phid_h + 0.5 * regt;
    const double pred_h = -(gs + 0.5 * (js + srs));
    const double rho_h = pred_h > 0.0 ? (st.phi_u - phi_h) / pred_h : -INFINITY;
    if (V.rep) {
        V.rep[slice].hook_rho[st.k - 1] = rho_h;
        V.rep[slice].hook_pred[st.k - 1] = pred_h;
    }
    if (rho_h > P.eta && pred_h >= st.pred) {
        st.hook_keep = 1;
        st.final_slot = SLOT_PHI_DATA_H;
        if (V.rep) V.rep[slice].hook_accepted[st.k - 1] = 1;
    }
}

// Accept: u <- u' (or the kept hook proposal, held in q) when the decision of
// this iteration accepted.
__global__ void __launch_bounds__(EW_THREADS) k_accept(VecArgs V)
{
    const int slice = blockIdx.y;
    const LMState& st = V.st[slice];
    if (st.done || !st.accepted) return;
    const int n2 = V.g.n * V.g.n;
    const size_t vo = (size_t)slice * V.vstride;
    const float* src = st.hook_keep ? V.q : V.ut;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        V.u[vo + m] = src[vo + m];
        V.u[vo + n2 + m] = src[vo + n2 + m];
    }
}

// End of an outer iteration: apply a stop decided in k_decide, or the end
// of the slice's max_outer iterations.
__global__ void k_commit(LMState* st, const LMParamsDev* prm, int n_slices)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    if (st[s].done_next || st[s].k >= prm[s].max_outer) st[s].done = 1;
}

// Slot pool: every slot finished (free slots are kept finished).
__global__ void k_pool_clear(LMState* st, int n_slices)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    LMState z = {};
    z.done = 1;
    st[s] = z;
}

// Slot pool: stop slot `slot` (its result was fetched, or it was cancelled).
__global__ void k_pool_release(LMState* st, int slot)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) st[slot].done = 1;
}

// Slot pool: 1 where a slot's solve has finished, else 0.
__global__ void k_pool_flags(const LMState* st, int* flags, int n_slices)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_slices) flags[s] = st[s].done ? 1 : 0;
}

// Regulariser energy of the returned maps with the alphas of iteration
// iters_run (partials for k_finish).
__global__ void __launch_bounds__(EW_THREADS) k_final_reg(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.y;
    const LMState& st = V.st[slice];
    const Geo& g = V.g;
    const int n = g.n, n2 = n * n;
    float af, am;
    alphas_at(V.prm[slice], st.k, af, am);
    const size_t vo = (size_t)slice * V.vstride;
    double reg = 0.0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n2) {
        const int r = m / n, c = m - r * n;
        reg = (double)af * grad2(V.u + vo, n, r, c) + (double)am * grad2(V.u + vo + n2, n, r, c);
        const LMParamsDev& P = V.prm[slice];
        if (P.prior_w) {
            const float ps = prior_scale(P, st.k);
            float wf, wm, rf0, rm0;
            prior_at(P, ps, m, wf, rf0);
            prior_at(P, ps, n2 + m, wm, rm0);
            const float df = V.u[vo + m] - rf0, dm = V.u[vo + n2 + m] - rm0;
            reg += (double)wf * ((double)df * df) + (double)wm * ((double)dm * dm);
        }
    }
    double s = block_sum(reg, sh);
    if (threadIdx.x == 0) slot_ptr(V.part, slice, SLOT_PHI_REG_U)[blockIdx.x] = s;
}

// Final report: Phi of the returned maps with the alphas of iteration
// iters_run; one block per slice, plus the scalar fields.
__global__ void __launch_bounds__(256) k_finish(VecArgs V)
{
    __shared__ double sh[16];
    const int slice = blockIdx.x;
    const LMState& st = V.st[slice];
    // Phi_data of the final iterate: the trial's if the last step was
    // accepted, else the linearisation point's.
    const int slot = st.final_slot;
    const double phid = sum_partials(slot_ptr(V.part, slice, slot), V.n_angle_parts, sh);
    const double reg = sum_partials(slot_ptr(V.part, slice, SLOT_PHI_REG_U), V.n_ew_blocks, sh);
    if (threadIdx.x != 0 || !V.rep) return;
    ReportDev& R = V.rep[slice];
    R.phi[st.k] = st.k == 0 ? NAN : 0.5 * phid + 0.5 * reg;
    R.scalars[0] = (double)st.status;
    R.scalars[1] = (double)st.k;
    R.scalars[2] = st.beta;
    R.scalars[3] = (double)st.stop_reason;
}

// ------------------------------------------------------------- launchers
// (host-callable wrappers used by the runtime; grid shapes are set there)
#define INST_MARCH(L, M, S) template __global__ void k_march<L, M, S>(MarchArgs);
#define INST_JVP(L, M, S) template __global__ void k_jvp_lin<L, M, S>(JvpArgs);
#define INST_JVP3(M, S) INST_JVP(IMG_HBM, M, S) INST_JVP(IMG_LDS, M, S) INST_JVP(IMG_BANDS, M, S)
#define INST_ALL(S)                                                                           \
    INST_MARCH(true, MARCH_FWD, S) INST_MARCH(true, MARCH_LIN, S) INST_MARCH(true, MARCH_TRIAL, S) \
    INST_MARCH(false, MARCH_FWD, S) INST_MARCH(false, MARCH_LIN, S)                           \
    INST_MARCH(false, MARCH_TRIAL, S)                                                         \
    INST_JVP3(JVP_PLAIN, S) INST_JVP3(JVP_NORMAL, S) INST_JVP3(JVP_SQNORM, S)                  \
    template __global__ void k_vjp_lin<S, false>(VjpArgs, const float4*, const int2*);                                    \
    template __global__ void k_pack<S>(Geo, PairSrc, const double*, void*, long long, const LMState*);
INST_ALL(F32S)
INST_ALL(BF16S)
INST_ALL(F32DR)
// the quarter-turn fold; not with a depth response (one staged angle only)
template __global__ void k_vjp_lin<F32S, true>(VjpArgs, const float4*, const int2*);
template __global__ void k_vjp_lin<BF16S, true>(VjpArgs, const float4*, const int2*);

}  // namespace pget
