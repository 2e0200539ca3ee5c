// Host runtime and C ABI of libpget: plans (geometry tables), workspace
// layout, launch shapes, and the device-resident Levenberg-Marquardt loop.
#include "pget.h"
#include "pget_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <vector>


using namespace pget;

struct pget_plan {
    pget_geometry geom;
    Geo g;
    Tables t;
    void* table_mem;     // one device allocation holding every table
    float* depth_mem = nullptr;   // per-sample depth factor (set on demand)
    float* resp_mem = nullptr;    // depth response: alpha per sample, then the far taps
    bool bf16;           // BF16 storage of staged maps and per-sample weights
    size_t px_bytes;     // bytes of one staged map pair (8 FP32, 4 BF16)
    size_t w_bytes;      // bytes of one per-sample weight pair
    bool lds_img;        // the FP32 map pair of the ray march fits in LDS
    bool jvp_lds;        // the map pair of the Jacobian product (storage type) fits in LDS
    size_t op_lds_bytes; // dynamic LDS of k_march
    int op_threads;      // threads per block of k_march
    size_t img_lds;      // LDS bytes of the staged map pair (0 if not staged)
    int jvp_bands;       // k_jvp_lin walks the pair in this many bands of rows (1: none)
    int jvp_band_h;      // top bordered rows per band
    int band_cand;       // bands the pair would take when staged in LDS (1: whole pair fits or none)
    int band_h_cand;
    size_t band_img_lds; // LDS bytes of one staged band
    bool band_staging;   // set by pget_plan_set_band_staging
    int max_japb;        // most angle slots per k_jvp_lin block that fit in LDS
    int max_japb_dr;     // the same with a depth response (three rows per slot)
    int vjp_resident_dr; // k_vjp_lin blocks per compute unit with a depth response
    int tiles_x;         // VJP tiles per edge
    int device;
    int n_cu;            // compute units of the device
    int vjp_resident;    // k_vjp_lin blocks resident per compute unit
    int64_t support;     // lattice samples inside the support
    std::vector<std::array<int, 3>> tuned;   // (batch, japb, vjp groups) picked by pget_autotune
};

// Scratch of the allocation-free forward map (pget_forward_noalloc): the
// zero-bordered map pair ((N + 2)^2 float2) that the ray march reads when the
// pair does not fit in LDS; at most 514^2 * 8 B for N = 512.  Each device
// the library runs on holds its own copy for the life of the process.  Host
// code uses only the device address looked up per device (g_scratch), never
// this name.
constexpr size_t NOALLOC_SCRATCH_BYTES = 2304u * 1024u;   // 2.25 MiB
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static void* g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mutex;

// Device address of `scratch` on the current device `device`, looked up on
// the first call for that device (plan creation is the set-up call).
static pget_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= MAX_DEVICES) return PGET_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PGET_ERR_HIP;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return PGET_OK;
}

static bool g_use_graphs = true;

// Instantiated solver sequences, keyed by workspace and the groups solved.
struct GraphKey {
    void* ws;
    std::vector<std::array<long long, 6>> groups;   // plan, batch, outer, cg, beta0 | trace << 1 | sgp << 2, offset
    bool operator==(const GraphKey& o) const { return ws == o.ws && groups == o.groups; }
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    unsigned long long used;   // last replay (a counter), for eviction
};
static std::vector<GraphEntry> g_graphs;
static unsigned long long g_graph_clock = 0;
// Executable graphs kept at once; the least recently replayed one is
// destroyed to make room (a caller that passes a fresh workspace per solve
// pays a capture per call but no growing set of graphs).
constexpr size_t GRAPH_CACHE = 32;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e__ = (expr);                       \
        if (e__ != hipSuccess) return PGET_ERR_HIP;    \
    } while (0)

bool geometry_ok(const pget_geometry* g)
{
    if (!g) return false;
    // N <= 512 and n_angles <= 1024 keep every reducing launch within
    // SLOT_WIDTH blocks per slice
    if (g->n < 2 || g->n > 512) return false;
    if (g->n_angles < 1 || g->n_angles > SLOT_WIDTH) return false;
    if (g->n_bins < 1 || g->n_bins > 8192) return false;
    if (!(g->bin_size >= 1.0) || !(g->step >= 1.0)) return false;   // <= 3 gather candidates per axis
    if (!(g->psf_sigma >= 0.0) || !(g->atten_scale > 0.0)) return false;
    if (!isfinite(g->angle0) || !isfinite(g->arc)) return false;
    if (g->psf_radius > 32) return false;
    if (g->psf_sigma > 0.0 && g->psf_radius < 0 && ceil(3.0 * g->psf_sigma) > 32.0) return false;
    return true;
}

int half_width(const pget_geometry* g)
{
    if (g->psf_sigma <= 0.0) return 0;
    if (g->psf_radius >= 0) return g->psf_radius;
    return (int)ceil(3.0 * g->psf_sigma);
}

// Dynamic LDS of a k_jvp_lin block of `japb` angle slots: the staged map
// pair, and per sinogram row z and K z (plus, with a depth response, the far
// part of z, and alpha per sample).
size_t jvp_lds_for(const pget_plan* P, int japb, int img)
{
    const size_t rows = P->t.resp ? 3 : 2;
    const size_t alpha = P->t.resp ? (size_t)P->g.n_t * sizeof(float) : 0;
    return (img == IMG_HBM ? 0 : P->img_lds) + rows * (size_t)japb * (P->g.paired ? 2 : 1) * P->g.n_bins * sizeof(float) +
           alpha;
}
int max_japb_of(const pget_plan* P) { return P->t.resp ? P->max_japb_dr : P->max_japb; }

// Fewest angle slots per product block for which staging the map pair in
// bands pays: every block stages all its bands, so with fewer slots the
// bordered copy in HBM, read through the caches, is cheaper (measured at
// 256^2: 5 slots per block, batch 15, 1052 ms per solve with bands against
// 1017 from HBM; 6 slots, batch 64, 3.05 against 3.37 ms per product).
constexpr int BAND_MIN_SLOTS = 6;

// Launch shapes for a batch of `batch` slices.
struct Shapes {
    int apb;          // angles per block of k_march
    int n_op_blocks;  // blocks per slice of k_march
    int japb;         // angle slots per block of k_jvp_lin
    int n_jvp_blocks; // blocks per slice of k_jvp_lin
    int jvp_threads;
    size_t jvp_lds;
    int jvp_img;      // where k_jvp_lin reads the direction (IMG_*)
    int groups;       // blocks per tile and slice of the adjoint gather
    int fine;         // fine angle groups of the gather (plan only)
    int spf;          // angle slots per fine group
    int gs;           // fine groups per super group (plan only)
    int fpb;          // fine groups per gather block: 1 or a multiple of gs
    int super_out;    // the gather writes super-group partials (else fine ones)
    int n_part;       // partial images per slice the gather writes
    int gfold;        // partials per super group in the consumer's sum
    int n_vjp_blocks; // blocks per slice of k_vjp_lin
    int n_ew_blocks;  // blocks per slice of the element-wise kernels
};

// Angle slots of the adjoint gather: one slot takes an angle with its mirror
// (paired) and the quarter-turn pair (quad; not with a depth response, whose
// far sums leave no registers for a second staged angle).
int vjp_slots(const pget_plan* P)
{
    const Geo& g = P->g;
    return (g.quad && !P->t.resp) ? g.n_angles / 4 : g.paired ? g.n_angles / 2 : g.n_angles;
}

// Angle groups of the adjoint gather.  The angle slots are cut into fine
// groups of spf consecutive slots (about FINE_GROUPS of them), and runs of gs
// fine groups form super groups.  A pixel's value is the sum of its slots in
// order within a fine group, of the fine groups in order within a super
// group, and of the super groups in order: fine and super groups depend on
// the plan alone, so a slice gets the same bits alone, in a batch or in a
// mixed call.  A launch either runs one fine group per block (small batches:
// many blocks) and leaves the folds to the consumer, or whole super groups
// per block (large batches: few partial images).
constexpr int FINE_GROUPS = 32;
constexpr int REF_BATCH = 64;   // the batch the super-group size is chosen for

// Launch rounds times the work of one block (its angle slots plus about one
// slot of fixed cost), counted against the resident gather blocks.
double gather_cost(const pget_plan* P, int batch, int fine, int spf, int fpb)
{
    const long long resident =
        (long long)P->n_cu * std::max(1, P->t.resp ? P->vjp_resident_dr : P->vjp_resident);
    const int c = (fine + fpb - 1) / fpb;
    const long long blocks = (long long)P->tiles_x * P->tiles_x * batch * c;
    const double rounds = (double)((blocks + resident - 1) / resident);
    return rounds * ((double)(std::min(fpb, fine) * spf) + 1.0);
}

void fine_groups(const pget_plan* P, int& fine, int& spf, int& gs)
{
    const int vslots = vjp_slots(P);
    spf = std::max(1, (vslots + FINE_GROUPS - 1) / FINE_GROUPS);
    fine = std::max(1, (vslots + spf - 1) / spf);
    gs = 1;
    double best = 1e30;
    for (int f = 1; f <= fine; ++f) {
        const double cost = gather_cost(P, REF_BATCH, fine, spf, f);
        if (cost < best * (1.0 - 1e-9)) { best = cost; gs = f; }
    }
}

// Gather blocks per tile and slice that run `fpb` fine groups each.
inline int coarse_of(int fine, int fpb) { return (fine + fpb - 1) / fpb; }

// Candidate fine groups per block: 1, or whole super groups.
std::vector<int> fpb_candidates(int fine, int gs)
{
    std::vector<int> c{1};
    for (int f = gs; f < fine + gs; f += gs)
        if (f > 1) c.push_back(f);
    return c;
}

// The gather's block count and output layout for `fpb` fine groups per block.
void set_fpb(Shapes& s, int fpb)
{
    // blocks never straddle a super group: whole super groups (or all fine
    // groups in one block), else one fine group each
    s.fpb = std::max(1, std::min(fpb, s.fine));
    const bool whole = s.fpb % s.gs == 0 || s.fpb == s.fine;
    if (!whole) s.fpb = 1;
    s.groups = coarse_of(s.fine, s.fpb);
    s.super_out = (s.fpb % s.gs == 0 || s.fpb == s.fine) ? 1 : 0;
    s.n_part = s.super_out ? coarse_of(s.fine, s.gs) : s.fine;
    s.gfold = s.super_out ? 1 : s.gs;
}

// Product shape of `japb` angle slots per block.
void set_japb(const pget_plan* P, Shapes& s, int japb)
{
    const int slots = P->g.paired ? P->g.n_angles / 2 : P->g.n_angles;
    s.japb = std::max(1, std::min(max_japb_of(P), japb));
    s.n_jvp_blocks = (slots + s.japb - 1) / s.japb;
    s.jvp_threads = std::min(16, s.japb * P->g.n_groups) * WAVE;
    s.jvp_img = !P->jvp_lds ? IMG_HBM : P->jvp_bands == 1 ? IMG_LDS : s.japb >= BAND_MIN_SLOTS ? IMG_BANDS : IMG_HBM;
    s.jvp_lds = jvp_lds_for(P, s.japb, s.jvp_img);
}

Shapes shapes_for(const pget_plan* P, int batch)
{
    Shapes s;
    const int cus = P->n_cu;
    // enough blocks to cover the chip twice; more angles per block when the
    // batch already does (the staged map is then reused across angles)
    int want = std::max(1, (P->g.n_angles * batch) / (4 * cus));
    s.apb = std::min(8, want);
    s.n_op_blocks = (P->g.n_angles + s.apb - 1) / s.apb;
    const int slots = P->g.paired ? P->g.n_angles / 2 : P->g.n_angles;
    int japb = std::max(1, (slots * batch) / (2 * cus));
    if (P->jvp_bands == 1) {
        // The map pair read whole, from LDS or from the bordered HBM copy: a
        // product block gains nothing from a second one sharing its CU
        // (measured), so a launch takes about ceil(blocks / CUs) rounds of
        // (slots per block + c0) slot times, c0 the per-block cost of staging
        // the map (2 slot times) or, reading the HBM copy, of the epilogue
        // (0.5); the fewest slots that reach the lowest cost win.  Measured
        // (LM solve of 15 x 30, slots per block from blocks enough to fill
        // the chip twice -> this rule): in LDS, 64^2 x 12 slices 61.3 -> 51.3
        // ms (4 -> 9 slots), 96^2 x 13 130.0 -> 113.9 (4 -> 10), 128^2 x 13
        // 220.5 -> 207.7 (4 -> 5), 128^2 x 8 137.2 -> 121.4 (2 -> 6), 128^2 x
        // 4 84.3 -> 64.4 (1 -> 3), 64^2 x 64 at 120 angles (15 x 20) 67.5 ->
        // 60.0 (7 -> 15), 128^2 x 64 and one slice unchanged; from the HBM
        // copy, 256^2 x 15 1026 -> 918 (5 -> 11), 192^2 x 11 417 -> 400 (3 ->
        // 8), 192^2 x 4 163 -> 156 and 256^2 x 4 257 -> 254 (1 -> 3), 64
        // slices of 192^2 2172 -> 2105 and of 256^2 3724 -> 3619 (16 -> 15).
        // Plans with band staging keep the chip-twice rule.
        const double c0 = P->jvp_lds ? 2.0 : 0.5;
        double best = 1e30;
        for (int j = 1; j <= max_japb_of(P); ++j) {
            const long long blocks = (long long)batch * ((slots + j - 1) / j);
            const double cost = (double)((blocks + cus - 1) / cus) * (j + c0);
            if (cost < best * (1.0 - 1e-9)) {
                best = cost;
                japb = j;
            }
        }
    }
    set_japb(P, s, japb);
    // blocks of the gather: the fewest launch rounds times the work of one
    // block (its angle slots plus about one slot of fixed cost), counted
    // against the resident blocks.  Small batches run one fine group per
    // block to fill the chip.
    const int tiles = P->tiles_x * P->tiles_x;
    fine_groups(P, s.fine, s.spf, s.gs);
    int fpb = 1;
    double best = 1e30;
    for (int f : fpb_candidates(s.fine, s.gs)) {
        const double cost = gather_cost(P, batch, s.fine, s.spf, f);
        if (cost < best * (1.0 - 1e-9)) { best = cost; fpb = f; }
    }
    for (const auto& t : P->tuned)
        if (t[0] == batch) {
            set_japb(P, s, t[1]);
            fpb = t[2];
        }
    set_fpb(s, fpb);
    s.n_vjp_blocks = tiles * s.groups;
    s.n_ew_blocks = (P->g.n * P->g.n + EW_THREADS - 1) / EW_THREADS;
    return s;
}

// Workspace layout.  Every buffer is 256-byte aligned.
struct Layout {
    size_t wts, wq, tsum, sino_a, sino_b, ymeas, gpart_grad, gpart_cg, gimg, part;
    long long far_off;   // depth response: elements from a sinogram plane to its far plane
    size_t u, ut, s, x, r, p, q, grad, fmask, state, params, repdev, reparr;
    size_t total;
};

Layout layout_for(const pget_plan* P, int op, int batch, const Shapes& sh, int max_outer, int n_cg)
{
    const Geo& g = P->g;
    Layout L = {};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    const size_t B = (size_t)batch;
    const size_t n2 = (size_t)g.n * g.n;
    const size_t sino = (size_t)g.n_angles * g.n_bins;
    const size_t lat = (size_t)P->support;   // compacted per-sample arrays: in-support samples only
    // with a depth response the ray totals and the blurred cotangents have a
    // far plane B * sino elements after the near one, and the far prefix
    // sums their own per-sample array
    const size_t planes = P->t.resp ? 2 : 1;
    L.far_off = (long long)(B * sino);
    if (op != PGET_OP_FORWARD) {
        L.wts = take(B * lat * P->w_bytes);
        if (P->t.resp) L.wq = take(B * lat * sizeof(float));
        L.tsum = take(planes * B * sino * sizeof(float));
    }
    L.sino_a = take(planes * B * sino * sizeof(float));
    L.sino_b = take(planes * B * sino * sizeof(float));
    // the bordered copy in HBM: for the march or for a product that does not
    // stage the whole pair in LDS
    L.gimg = (P->lds_img && P->jvp_lds && P->jvp_bands == 1) ? 0 : take(B * (size_t)g.pitch * g.pitch * sizeof(float2));
    L.part = take(B * (size_t)N_SLOTS * SLOT_WIDTH * sizeof(double));
    if (op == PGET_OP_VJP || op == PGET_OP_LM) L.gpart_cg = take((size_t)sh.fine * B * 2 * n2 * sizeof(float));
    if (op == PGET_OP_LM) {
        L.gpart_grad = take((size_t)sh.fine * B * 2 * n2 * sizeof(float));
        L.ymeas = take(B * sino * sizeof(float));
        L.u = take(B * 2 * n2 * sizeof(float));
        L.ut = take(B * 2 * n2 * sizeof(float));
        L.s = take(B * 2 * n2 * sizeof(float));
        L.x = take(B * 2 * n2 * sizeof(float));
        L.r = take(B * 2 * n2 * sizeof(float));
        L.p = take(B * 2 * n2 * sizeof(float));
        L.q = take(B * 2 * n2 * sizeof(float));
        L.grad = take(B * 2 * n2 * sizeof(float));
        L.fmask = take(B * 2 * n2);
        L.state = take(B * sizeof(LMState));
        L.params = take(B * sizeof(LMParamsDev));
        L.repdev = take(B * sizeof(ReportDev));
        const size_t per = (size_t)(max_outer + 1) * 8 * sizeof(double) + 2 * (size_t)max_outer +
                           (size_t)max_outer * n_cg * sizeof(double) + 4 * sizeof(double) + 64;
        L.reparr = take(B * align_up(per));
    }
    L.total = off;
    return L;
}

inline char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// ---- optional launch timing (pget_timing_enable)
struct TimingRec {
    int cls;
    hipEvent_t start, stop;
};
struct Timing {
    int classes = 0;
    int capacity = 0;
    std::vector<hipEvent_t> pool;   // 2 * capacity events
    std::vector<TimingRec> recs;
} g_timing;

// RAII bracket around one kernel launch of class `cls` on stream `s`.
struct Timed {
    TimingRec* rec = nullptr;
    hipStream_t s;
    Timed(int cls, hipStream_t stream) : s(stream)
    {
        if (!(g_timing.classes & (1 << cls))) return;
        if ((int)g_timing.recs.size() >= g_timing.capacity) return;
        const size_t k = g_timing.recs.size();
        g_timing.recs.push_back(TimingRec{cls, g_timing.pool[2 * k], g_timing.pool[2 * k + 1]});
        rec = &g_timing.recs.back();
        (void)hipEventRecord(rec->start, s);
    }
    ~Timed()
    {
        if (rec) (void)hipEventRecord(rec->stop, s);
    }
};

Tables tables_of(const pget_plan* P) { return P->t; }

template <bool LDS, int M>
void launch_march(const pget_plan* P, const MarchArgs& A, int blocks, int batch, hipStream_t s)
{
    Timed t(PGET_KC_MARCH, s);
    if (P->t.resp)   // one more row of ray sums (the far part)
        hipLaunchKernelGGL((k_march<LDS, M, F32DR>), dim3(blocks, batch), dim3(P->op_threads),
                           P->op_lds_bytes + P->g.n_bins * sizeof(float), s, A);
    else if (P->bf16)
        hipLaunchKernelGGL((k_march<LDS, M, BF16S>), dim3(blocks, batch), dim3(P->op_threads), P->op_lds_bytes,
                           s, A);
    else
        hipLaunchKernelGGL((k_march<LDS, M, F32S>), dim3(blocks, batch), dim3(P->op_threads), P->op_lds_bytes,
                           s, A);
}
template <int M>
void march(const pget_plan* P, const MarchArgs& A, int blocks, int batch, hipStream_t s)
{
    if (P->lds_img) launch_march<true, M>(P, A, blocks, batch, s);
    else launch_march<false, M>(P, A, blocks, batch, s);
}
template <int LDS, int M>
void launch_jvp(const pget_plan* P, const JvpArgs& A, const Shapes& sh, int batch, hipStream_t s)
{
    Timed t(PGET_KC_JVP, s);
    if (P->t.resp)
        hipLaunchKernelGGL((k_jvp_lin<LDS, M, F32DR>), dim3(sh.n_jvp_blocks, batch), dim3(sh.jvp_threads),
                           sh.jvp_lds, s, A);
    else if (P->bf16)
        hipLaunchKernelGGL((k_jvp_lin<LDS, M, BF16S>), dim3(sh.n_jvp_blocks, batch), dim3(sh.jvp_threads),
                           sh.jvp_lds, s, A);
    else
        hipLaunchKernelGGL((k_jvp_lin<LDS, M, F32S>), dim3(sh.n_jvp_blocks, batch), dim3(sh.jvp_threads),
                           sh.jvp_lds, s, A);
}
template <int M>
void jvp(const pget_plan* P, const JvpArgs& A, const Shapes& sh, int batch, hipStream_t s)
{
    if (sh.jvp_img == IMG_HBM) launch_jvp<IMG_HBM, M>(P, A, sh, batch, s);
    else if (sh.jvp_img == IMG_BANDS) launch_jvp<IMG_BANDS, M>(P, A, sh, batch, s);
    else launch_jvp<IMG_LDS, M>(P, A, sh, batch, s);
}

// The grid is (tiles * V.groups, batch): the kernel decodes (slice, group,
// tile) from the linear block id with exactly these extents.
void launch_vjp(const pget_plan* P, const VjpArgs& V, int batch, hipStream_t s)
{
    const dim3 grid(P->tiles_x * P->tiles_x * V.groups, batch), block(VJP_THREADS);
    if (P->t.resp) {
        hipLaunchKernelGGL((k_vjp_lin<F32DR, false>), grid, block, 0, s, V, V.t.trig, V.t.gcol);
    } else if (P->bf16) {
        if (P->g.quad) hipLaunchKernelGGL((k_vjp_lin<BF16S, true>), grid, block, 0, s, V, V.t.trig, V.t.gcol);
        else hipLaunchKernelGGL((k_vjp_lin<BF16S, false>), grid, block, 0, s, V, V.t.trig, V.t.gcol);
    } else {
        if (P->g.quad) hipLaunchKernelGGL((k_vjp_lin<F32S, true>), grid, block, 0, s, V, V.t.trig, V.t.gcol);
        else hipLaunchKernelGGL((k_vjp_lin<F32S, false>), grid, block, 0, s, V, V.t.trig, V.t.gcol);
    }
}

// Global bordered copy of a map pair: FP32 for the ray march (jvp_store =
// false), the plan's storage for the Jacobian product (jvp_store = true).
void pack(const pget_plan* P, const PairSrc& src, const double* part, void* out, int batch,
          const LMState* st, hipStream_t s, bool jvp_store = false)
{
    const int total = P->g.pitch * P->g.pitch;
    const int blocks = std::min(1024, (total + 255) / 256);
    Timed t(PGET_KC_CONTROL, s);
    if (P->bf16 && jvp_store)
        hipLaunchKernelGGL(k_pack<BF16S>, dim3(blocks, batch), dim3(256), 0, s, P->g, src, part, out,
                           (long long)total, st);
    else
        hipLaunchKernelGGL(k_pack<F32S>, dim3(blocks, batch), dim3(256), 0, s, P->g, src, part, out,
                           (long long)total, st);
}

void fill_zero(void* p, size_t bytes, hipStream_t s)
{
    const long long n4 = (long long)(bytes / 16);
    const int blocks = (int)std::min<long long>(4096, (n4 + 255) / 256);
    if (n4 > 0) {
        Timed t_(PGET_KC_CONTROL, s);
        hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, reinterpret_cast<float4*>(p), n4);
    }
}

// Block and group counts of a gather launch.
void set_groups(VjpArgs& V, const Shapes& sh)
{
    V.groups = sh.groups;
    V.fine = sh.fine;
    V.spf = sh.spf;
    V.fpb = sh.fpb;
    V.gs = sh.gs;
    V.super_out = sh.super_out;
}

PairSrc planar_src(const float* f, const float* mu, long long stride)
{
    PairSrc s = {};
    s.af = f;
    s.am = mu;
    s.stride = stride;
    s.kind = 0;
    return s;
}

// Where the Jacobian product reads the direction, and the LDS limits that
// follow: the whole bordered pair staged in LDS when it fits; else, with
// band staging on and bands possible, the plan's bands (staged by blocks of
// enough angle slots, walked from the HBM copy by the others); else the HBM
// copy in one pass.
void apply_jvp_lds(pget_plan* P, size_t jimg_bytes, size_t per_slot)
{
    const size_t lds_budget = 160 * 1024 - 2048;
    const bool whole = jimg_bytes + per_slot <= lds_budget;
    const bool bands = !whole && P->band_staging && P->band_cand > 1;
    P->jvp_lds = whole || bands;
    P->img_lds = whole ? jimg_bytes : bands ? P->band_img_lds : 0;
    P->jvp_bands = bands ? P->band_cand : 1;
    P->jvp_band_h = bands ? P->band_h_cand : P->g.n + 1;
    P->max_japb = (int)std::min<size_t>(16, (lds_budget - P->img_lds) / per_slot);
    const size_t alpha_bytes = (size_t)P->g.n_t * sizeof(float);
    P->max_japb_dr = lds_budget >= P->img_lds + alpha_bytes
                         ? (int)std::min<size_t>(16, (lds_budget - P->img_lds - alpha_bytes) / (per_slot / 2 * 3))
                         : 0;
}

}  // namespace

extern "C" {

const char* pget_status_string(pget_status st)
{
    switch (st) {
    case PGET_OK: return "ok";
    case PGET_ERR_INVALID_ARG: return "invalid argument";
    case PGET_ERR_HIP: return "HIP runtime error";
    case PGET_ERR_WORKSPACE: return "workspace missing or too small";
    case PGET_ERR_NONFINITE: return "non-finite value in the solver";
    case PGET_ERR_UNSUPPORTED: return "unsupported geometry";
    }
    return "unknown status";
}

pget_status pget_plan_create(const pget_geometry* geom, pget_storage storage, pget_plan** out)
{
    if (!out) return PGET_ERR_INVALID_ARG;
    *out = nullptr;
    if (!geometry_ok(geom)) return PGET_ERR_INVALID_ARG;
    if (storage != PGET_FP32 && storage != PGET_BF16) return PGET_ERR_UNSUPPORTED;
    pget_plan* P = new (std::nothrow) pget_plan();
    if (!P) return PGET_ERR_HIP;
    P->geom = *geom;
    P->bf16 = storage == PGET_BF16;
    P->px_bytes = P->bf16 ? 4 : 8;
    P->w_bytes = P->bf16 ? 4 : 8;
    Geo& g = P->g;
    g.n = geom->n;
    g.n_angles = geom->n_angles;
    g.n_bins = geom->n_bins;
    g.n_t = 2 * (int)ceil(((double)geom->n / sqrt(2.0) + 1.0) / geom->step);
    g.K = half_width(geom);
    g.pitch = g.n + 2;
    g.n_groups = (g.n_bins + RG - 1) / RG;
    g.step = (float)geom->step;
    g.bin_size = (float)geom->bin_size;
    g.t_off = 0.5f * (float)(g.n_t - 1);
    g.s_off = 0.5f * (float)(g.n_bins - 1);
    g.half = 0.5f * (float)(g.n - 1);
    g.c_att = (float)geom->atten_scale;
    g.kq = (float)(-geom->atten_scale * geom->step * geom->step);
    g.ln2_scale = (float)(geom->atten_scale * geom->step * 1.4426950408889634);
    g.paired = (geom->n_angles % 2 == 0) && fabs(geom->arc - 2.0 * M_PI) <= 1e-12 * 2.0 * M_PI;
    g.quad = g.paired && geom->n_angles % 4 == 0 && geom->step == geom->bin_size &&
             (g.n_bins - g.n_t) % 2 == 0;
    g.rot_c = (g.n_t + g.n_bins) / 2 - 1;
    g.rot_d = (g.n_bins - g.n_t) / 2;

    // ---- tables in double precision, stored rounded to float
    const int na = g.n_angles, nb = g.n_bins, nt = g.n_t, ng = g.n_groups, K = g.K;
    std::vector<float4> trig(na);
    std::vector<float2> rbase((size_t)na * nb);
    std::vector<int2> clip((size_t)na * nb);
    std::vector<int2> grange((size_t)na * ng);
    std::vector<float> taps(2 * K + 1);
    const double half = 0.5 * (g.n - 1), soff = 0.5 * (nb - 1), toff = 0.5 * (nt - 1);
    for (int a = 0; a < na; ++a) {
        const double th = geom->angle0 + (double)a * geom->arc / (double)na;
        const double cs = cos(th), sn = sin(th);
        trig[a] = make_float4((float)(geom->step * cs), (float)(geom->step * sn), (float)cs, (float)sn);
        for (int grp = 0; grp < ng; ++grp) grange[(size_t)a * ng + grp] = make_int2(1, 0);
        for (int j = 0; j < nb; ++j) {
            const double s = ((double)j - soff) * geom->bin_size;
            const double cb = -s * sn + half, rbv = s * cs + half;
            rbase[(size_t)a * nb + j] = make_float2((float)cb, (float)rbv);
            int lo = nt, hi = -1;
            for (int i = 0; i < nt; ++i) {
                const double t = ((double)i - toff) * geom->step;
                const double col = cb + t * cs, row = rbv + t * sn;
                if (col > -1.0 && col < (double)g.n && row > -1.0 && row < (double)g.n) {
                    lo = std::min(lo, i);
                    hi = std::max(hi, i);
                }
            }
            if (hi < lo) { lo = 1; hi = 0; }
            clip[(size_t)a * nb + j] = make_int2(lo, hi);
        }
    }
    // A full turn with an even angle count: ray n_b-1-j of angle a + n/2
    // visits ray j's points in reverse; its clip range is taken from ray j's
    // (exact symmetry, whatever the rounding of the two FP64 tests), so that
    // a sample and its mirror are in the support together.
    if (g.paired)
        for (int a = 0; a < na / 2; ++a)
            for (int j = 0; j < nb; ++j) {
                const int2 c = clip[(size_t)a * nb + j];
                clip[(size_t)(a + na / 2) * nb + (nb - 1 - j)] =
                    c.y >= c.x ? make_int2(nt - 1 - c.y, nt - 1 - c.x) : make_int2(1, 0);
            }
    // ray offsets of the compacted per-sample arrays: a ray's in-support
    // samples contiguous, rays in (angle, bin) order, except that in paired
    // geometry ray (a + n_a/2, n_b-1-j) follows ray (a, j) (the adjoint then
    // finds the mirror's samples from the ray's own offset)
    std::vector<int> roff((size_t)na * nb);
    auto place = [&](size_t r) {
        const int2 c = clip[r];
        roff[r] = (int)std::min<int64_t>(P->support, INT32_MAX);
        if (c.y >= c.x) P->support += c.y - c.x + 1;
    };
    for (int a = 0; a < (g.paired ? na / 2 : na); ++a)
        for (int j = 0; j < nb; ++j) {
            place((size_t)a * nb + j);
            if (g.paired) place((size_t)(a + na / 2) * nb + (nb - 1 - j));
        }
    if (P->support >= ((int64_t)1 << 29)) {
        delete P;
        return PGET_ERR_UNSUPPORTED;   // the adjoint's byte offsets (8 B per sample) are 32-bit
    }
    // the groups' unions of clip ranges
    for (int a = 0; a < na; ++a)
        for (int j = 0; j < nb; ++j) {
            const int2 c = clip[(size_t)a * nb + j];
            if (c.y < c.x) continue;
            int2& gr = grange[(size_t)a * ng + j / RG];
            if (gr.y < gr.x) gr = c;
            else gr = make_int2(std::min(gr.x, c.x), std::max(gr.y, c.y));
        }
    // the adjoint's column table: (lo | len << 16, offset of sample 0); empty
    // rays (0, 0).  n_t <= 728 (n <= 512, step >= 1) fits 16 bits.
    std::vector<int2> gcol((size_t)na * nb);
    for (size_t r = 0; r < gcol.size(); ++r) {
        const int2 c = clip[r];
        gcol[r] = c.y >= c.x ? make_int2(c.x | ((c.y - c.x + 1) << 16), roff[r] - c.x) : make_int2(0, 0);
    }
    if (K == 0) taps[0] = 1.0f;
    else {
        std::vector<double> t(2 * K + 1);
        double sum = 0.0;
        for (int k = -K; k <= K; ++k) {
            t[k + K] = exp(-(double)(k * k) / (2.0 * geom->psf_sigma * geom->psf_sigma));
            sum += t[k + K];
        }
        for (int k = 0; k < 2 * K + 1; ++k) taps[k] = (float)(t[k] / sum);
    }
    size_t o_trig = 0;
    size_t o_rbase = align_up(o_trig + trig.size() * sizeof(float4));
    size_t o_clip = align_up(o_rbase + rbase.size() * sizeof(float2));
    size_t o_gr = align_up(o_clip + clip.size() * sizeof(int2));
    size_t o_taps = align_up(o_gr + grange.size() * sizeof(int2));
    size_t o_roff = align_up(o_taps + taps.size() * sizeof(float));
    size_t o_gcol = align_up(o_roff + roff.size() * sizeof(int));
    size_t total = align_up(o_gcol + gcol.size() * sizeof(int2));
    if (hipGetDevice(&P->device) != hipSuccess || hipMalloc(&P->table_mem, total) != hipSuccess) {
        delete P;
        return PGET_ERR_HIP;
    }
    char* base = static_cast<char*>(P->table_mem);
    bool ok = hipMemcpy(base + o_trig, trig.data(), trig.size() * sizeof(float4), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_rbase, rbase.data(), rbase.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_clip, clip.data(), clip.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_gr, grange.data(), grange.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_taps, taps.data(), taps.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_roff, roff.data(), roff.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + o_gcol, gcol.data(), gcol.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(P->table_mem);
        delete P;
        return PGET_ERR_HIP;
    }
    P->t.trig = reinterpret_cast<const float4*>(base + o_trig);
    P->t.rbase = reinterpret_cast<const float2*>(base + o_rbase);
    P->t.clip = reinterpret_cast<const int2*>(base + o_clip);
    P->t.grange = reinterpret_cast<const int2*>(base + o_gr);
    P->t.taps = reinterpret_cast<const float*>(base + o_taps);
    P->t.roff = reinterpret_cast<const int*>(base + o_roff);
    P->t.gcol = reinterpret_cast<const int2*>(base + o_gcol);
    P->t.depth = nullptr;
    P->t.resp = nullptr;
    P->t.taps_far = nullptr;

    // ---- launch shapes
    // the ray march stages the FP32 map pair; the Jacobian product stages the
    // pair in the storage type
    const size_t img_bytes = (size_t)g.pitch * g.pitch * sizeof(float2);
    const size_t jimg_bytes = (size_t)g.pitch * g.pitch * P->px_bytes;
    const size_t row_bytes = 2 * (size_t)nb * sizeof(float);
    const size_t lds_budget = 160 * 1024 - 2048;   // static shared arrays take the rest
    P->lds_img = img_bytes + row_bytes <= lds_budget;
    P->op_lds_bytes = (P->lds_img ? img_bytes : 0) + row_bytes;
    if (P->op_lds_bytes > lds_budget) {
        (void)hipFree(P->table_mem);
        delete P;
        return PGET_ERR_UNSUPPORTED;
    }
    P->op_threads = std::min(ng, 16) * WAVE;
    {
        const size_t per_slot = 2 * (size_t)(g.paired ? 2 : 1) * nb * sizeof(float);
        P->band_cand = 1;
        P->band_h_cand = g.n + 1;
        P->band_img_lds = 0;
        P->band_staging = false;
        if (jimg_bytes + per_slot > lds_budget) {
            // the pair in bands of bordered rows, leaving room for the rows
            // of four angle slots and a depth response's alpha table (with
            // a depth response, three rows per slot: fewer slots per block)
            const size_t row_px = (size_t)g.pitch * P->px_bytes;
            const size_t keep = 4 * per_slot + (size_t)nt * sizeof(float);
            if (lds_budget > keep + 9 * row_px) {
                const int h = (int)((lds_budget - keep) / row_px) - 1;   // staged rows h + 1
                const int bands = (g.n + 1 + h - 1) / h;
                // every band runs the block's items again: past 8 bands the
                // HBM copy read through the caches is kept
                if (bands <= 8) {
                    P->band_cand = bands;
                    P->band_h_cand = (g.n + 1 + bands - 1) / bands;
                    P->band_img_lds = (size_t)(P->band_h_cand + 1) * row_px;
                }
            }
        }
        apply_jvp_lds(P, jimg_bytes, per_slot);
        if (P->max_japb < 1) {
            (void)hipFree(P->table_mem);
            delete P;
            return PGET_ERR_UNSUPPORTED;
        }
    }
    {
        const int bytes = (int)lds_budget;
        bool attr_ok = true;
        {
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_FWD, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_LIN, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_TRIAL, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_PLAIN, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_NORMAL, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_SQNORM, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_FWD, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_LIN, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_TRIAL, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_PLAIN, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_NORMAL, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_SQNORM, F32S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_FWD, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_LIN, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_TRIAL, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_PLAIN, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_NORMAL, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_SQNORM, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_FWD, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_LIN, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_TRIAL, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_PLAIN, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_NORMAL, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_SQNORM, BF16S>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_FWD, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_LIN, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<true, MARCH_TRIAL, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_PLAIN, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_NORMAL, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<true, JVP_SQNORM, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_FWD, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_LIN, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_march<false, MARCH_TRIAL, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_PLAIN, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_NORMAL, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
            attr_ok &= hipFuncSetAttribute((const void*)k_jvp_lin<false, JVP_SQNORM, F32DR>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
        }
        if (!attr_ok) {
            (void)hipFree(P->table_mem);
            delete P;
            return PGET_ERR_HIP;
        }
    }
    {
        void* scr = nullptr;
        if (scratch_address(P->device, &scr) != PGET_OK) {
            (void)hipFree(P->table_mem);
            delete P;
            return PGET_ERR_HIP;
        }
    }
    P->tiles_x = (g.n + VT - 1) / VT;
    {
        int occ = 0, occ_dr = 0;
        const void* vk = g.quad ? (P->bf16 ? (const void*)k_vjp_lin<BF16S, true> : (const void*)k_vjp_lin<F32S, true>)
                                : (P->bf16 ? (const void*)k_vjp_lin<BF16S, false> : (const void*)k_vjp_lin<F32S, false>);
        const void* vk_dr = (const void*)k_vjp_lin<F32DR, false>;
        if (hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, vk, VJP_THREADS, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_dr, vk_dr, VJP_THREADS, 0) != hipSuccess) {
            (void)hipFree(P->table_mem);
            delete P;
            return PGET_ERR_HIP;
        }
        P->n_cu = std::max(1, P->n_cu);
        P->vjp_resident = std::max(1, occ);
        P->vjp_resident_dr = std::max(1, occ_dr);
    }
    *out = P;
    return PGET_OK;
}

// Captured solver sequences that launch kernels of this plan (their kernel
// arguments hold the plan's shapes and table pointers).
static void drop_graphs(const pget_plan* plan)
{
    for (size_t k = 0; k < g_graphs.size();) {
        bool uses = false;
        for (auto& gk : g_graphs[k].key.groups) uses |= gk[0] == (long long)(intptr_t)plan;
        if (uses) {
            (void)hipGraphExecDestroy(g_graphs[k].exec);
            g_graphs.erase(g_graphs.begin() + k);
        } else {
            ++k;
        }
    }
}

void pget_plan_destroy(pget_plan* plan)
{
    if (!plan) return;
    drop_graphs(plan);
    (void)hipFree(plan->table_mem);
    if (plan->depth_mem) (void)hipFree(plan->depth_mem);
    if (plan->resp_mem) (void)hipFree(plan->resp_mem);
    delete plan;
}

pget_status pget_plan_set_depth_response(pget_plan* plan, const double* alpha, int32_t n, const double* far_taps,
                                         int32_t n_taps)
{
    if (!plan) return PGET_ERR_INVALID_ARG;
    if (!alpha) {
        plan->t.resp = nullptr;
        plan->t.taps_far = nullptr;
        drop_graphs(plan);
        return PGET_OK;
    }
    const Geo& g = plan->g;
    if (n != g.n_t || !far_taps || n_taps != 2 * g.K + 1) return PGET_ERR_INVALID_ARG;
    std::vector<float> h((size_t)n + n_taps);
    for (int i = 0; i < n; ++i) {
        if (!(alpha[i] >= 0.0 && alpha[i] <= 1.0)) return PGET_ERR_INVALID_ARG;
        h[i] = (float)alpha[i];
    }
    for (int k = 0; k < n_taps; ++k) {
        // the adjoint applies the same taps: the response must be symmetric
        if (!isfinite(far_taps[k]) || far_taps[k] != far_taps[n_taps - 1 - k]) return PGET_ERR_INVALID_ARG;
        h[(size_t)n + k] = (float)far_taps[k];
    }
    // BF16 storage has no variant with the far sums; the extra LDS row must fit
    const size_t lds_budget = 160 * 1024 - 2048;
    if (plan->bf16 || plan->max_japb_dr < 1 || plan->op_lds_bytes + g.n_bins * sizeof(float) > lds_budget)
        return PGET_ERR_UNSUPPORTED;
    if (!plan->resp_mem && hipMalloc(&plan->resp_mem, h.size() * sizeof(float)) != hipSuccess) {
        plan->resp_mem = nullptr;
        return PGET_ERR_HIP;
    }
    if (hipMemcpy(plan->resp_mem, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return PGET_ERR_HIP;
    plan->t.resp = plan->resp_mem;
    plan->t.taps_far = plan->resp_mem + n;
    drop_graphs(plan);
    return PGET_OK;
}

pget_status pget_plan_set_depth_factor(pget_plan* plan, const double* depth, int32_t n)
{
    if (!plan) return PGET_ERR_INVALID_ARG;
    if (!depth) {
        plan->t.depth = nullptr;
        drop_graphs(plan);
        return PGET_OK;
    }
    if (n != plan->g.n_t) return PGET_ERR_INVALID_ARG;
    std::vector<float> d((size_t)n);
    for (int i = 0; i < n; ++i) {
        if (!(depth[i] > 0.0) || !isfinite(depth[i])) return PGET_ERR_INVALID_ARG;
        d[i] = (float)depth[i];
    }
    if (!plan->depth_mem && hipMalloc(&plan->depth_mem, (size_t)n * sizeof(float)) != hipSuccess) {
        plan->depth_mem = nullptr;
        return PGET_ERR_HIP;
    }
    if (hipMemcpy(plan->depth_mem, d.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return PGET_ERR_HIP;
    plan->t.depth = plan->depth_mem;
    drop_graphs(plan);
    return PGET_OK;
}

int32_t pget_plan_n_samples(const pget_plan* plan) { return plan ? plan->g.n_t : -1; }
int32_t pget_plan_psf_half_width(const pget_plan* plan) { return plan ? plan->g.K : -1; }
int64_t pget_plan_support_samples(const pget_plan* plan) { return plan ? plan->support : -1; }

pget_status pget_plan_set_band_staging(pget_plan* P, int32_t enable)
{
    if (!P) return PGET_ERR_INVALID_ARG;
    const bool on = enable != 0 && P->band_cand > 1;
    if (on == P->band_staging) return PGET_OK;
    const size_t jimg_bytes = (size_t)P->g.pitch * P->g.pitch * P->px_bytes;
    const size_t per_slot = 2 * (size_t)(P->g.paired ? 2 : 1) * P->g.n_bins * sizeof(float);
    P->band_staging = on;
    apply_jvp_lds(P, jimg_bytes, per_slot);
    if (P->max_japb < 1 || (P->t.resp && P->max_japb_dr < 1)) {
        P->band_staging = !on;
        apply_jvp_lds(P, jimg_bytes, per_slot);
        return PGET_ERR_UNSUPPORTED;
    }
    // captured solver sequences and tuned shapes assumed the old limits
    drop_graphs(P);
    P->tuned.clear();
    return PGET_OK;
}

int32_t pget_plan_jvp_bands(const pget_plan* P) { return P ? P->jvp_bands : -1; }

size_t pget_workspace_bytes(const pget_plan* plan, int32_t op, int32_t batch)
{
    if (!plan || batch < 1 || op < PGET_OP_FORWARD || op > PGET_OP_LM) return 0;
    if (op != PGET_OP_LM && batch != 1) return 0;
    Shapes sh = shapes_for(plan, batch);
    // report arrays are sized for the largest supported solve
    Layout L = layout_for(plan, op, batch, sh, 256, 256);
    return L.total;
}

}  // extern "C"

// The forward map with the bordered copy of the map pair (used when the pair
// does not fit in LDS) in `gimg`.
static pget_status forward_into(const pget_plan* P, const float* f, const float* mu, float* y, void* gimg,
                                hipStream_t stream)
{
    Shapes sh = shapes_for(P, 1);
    MarchArgs A = {};
    A.g = P->g;
    A.t = P->t;
    A.src = planar_src(f, mu, 0);
    A.sino_stride = (long long)P->g.n_angles * P->g.n_bins;
    A.yout = y;
    A.angles_per_block = sh.apb;
    if (!P->lds_img) {
        A.gimg = gimg;
        pack(P, A.src, nullptr, gimg, 1, nullptr, stream);
    }
    march<MARCH_FWD>(P, A, sh.n_op_blocks, 1, stream);
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

extern "C" {

pget_status pget_forward(const pget_plan* P, const float* f, const float* mu, float* y, void* ws,
                         hipStream_t stream)
{
    if (!P || !f || !mu || !y) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    Shapes sh = shapes_for(P, 1);
    Layout L = layout_for(P, PGET_OP_FORWARD, 1, sh, 256, 256);
    return forward_into(P, f, mu, y, at(ws, L.gimg), stream);
}

pget_status pget_forward_noalloc(const pget_plan* P, const float* f, const float* mu, float* y,
                                 hipStream_t stream)
{
    if (!P || !f || !mu || !y) return PGET_ERR_INVALID_ARG;
    const size_t need = P->lds_img ? 0 : (size_t)P->g.pitch * P->g.pitch * sizeof(float2);
    if (need > NOALLOC_SCRATCH_BYTES) return PGET_ERR_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PGET_ERR_HIP;
    if (dev != P->device) return PGET_ERR_INVALID_ARG;   // the plan's tables live on its device
    void* scr = nullptr;
    pget_status rc = scratch_address(dev, &scr);
    if (rc != PGET_OK) return rc;
    return forward_into(P, f, mu, y, scr, stream);
}

// Linearise at (f, mu): per-sample weights and ray totals into the workspace.
static void linearise(const pget_plan* P, const float* f, const float* mu, float* y_or_null,
                      void* ws, const Layout& L, const Shapes& sh, hipStream_t stream)
{
    MarchArgs A = {};
    A.g = P->g;
    A.t = P->t;
    A.src = planar_src(f, mu, 0);
    A.wts = at(ws, L.wts);
    A.tsum = reinterpret_cast<float*>(at(ws, L.tsum));
    A.wq = P->t.resp ? reinterpret_cast<float*>(at(ws, L.wq)) : nullptr;
    A.far_off = L.far_off;
    A.sino_stride = (long long)P->g.n_angles * P->g.n_bins;
    A.wts_stride = P->support;
    A.yout = y_or_null;
    A.angles_per_block = sh.apb;
    if (!P->lds_img) {
        A.gimg = at(ws, L.gimg);
        pack(P, A.src, nullptr, at(ws, L.gimg), 1, nullptr, stream);
    }
    march<MARCH_LIN>(P, A, sh.n_op_blocks, 1, stream);
}

pget_status pget_jvp(const pget_plan* P, const float* f, const float* mu, const float* vf,
                     const float* vmu, float* jv, float* y_or_null, void* ws, hipStream_t stream)
{
    if (!P || !f || !mu || !vf || !vmu || !jv) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    Shapes sh = shapes_for(P, 1);
    Layout L = layout_for(P, PGET_OP_JVP, 1, sh, 256, 256);
    linearise(P, f, mu, y_or_null, ws, L, sh, stream);
    JvpArgs A = {};
    A.g = P->g;
    A.t = P->t;
    A.bands = P->jvp_bands;
    A.band_h = P->jvp_band_h;
    A.src = planar_src(vf, vmu, 0);
    A.wts = at(ws, L.wts);
    A.tsum = reinterpret_cast<float*>(at(ws, L.tsum));
    A.wq = P->t.resp ? reinterpret_cast<const float*>(at(ws, L.wq)) : nullptr;
    A.far_off = L.far_off;
    A.sino_stride = (long long)P->g.n_angles * P->g.n_bins;
    A.wts_stride = P->support;
    A.out = jv;
    A.angles_per_block = sh.apb;
    if (sh.jvp_img == IMG_HBM) {
        A.gimg = at(ws, L.gimg);
        pack(P, A.src, nullptr, at(ws, L.gimg), 1, nullptr, stream, true);
    }
    A.angles_per_block = sh.japb;
    jvp<JVP_PLAIN>(P, A, sh, 1, stream);
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

pget_status pget_vjp(const pget_plan* P, const float* f, const float* mu, const float* w, float* gf,
                     float* gmu, void* ws, hipStream_t stream)
{
    if (!P || !f || !mu || !w || !gf || !gmu) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    Shapes sh = shapes_for(P, 1);
    Layout L = layout_for(P, PGET_OP_VJP, 1, sh, 256, 256);
    linearise(P, f, mu, nullptr, ws, L, sh, stream);
    float* wt = reinterpret_cast<float*>(at(ws, L.sino_a));
    {
        Timed t_(PGET_KC_CONTROL, stream);
        hipLaunchKernelGGL(k_psf, dim3(P->g.n_angles), dim3(256), P->g.n_bins * sizeof(float), stream, P->g,
                           P->t.taps, w, wt);
        if (P->t.resp)   // the cotangent seen through the far response (symmetric taps)
            hipLaunchKernelGGL(k_psf, dim3(P->g.n_angles), dim3(256), P->g.n_bins * sizeof(float), stream, P->g,
                               P->t.taps_far, w, wt + L.far_off);
    }
    VjpArgs V = {};
    V.g = P->g;
    V.t = P->t;
    V.wts = at(ws, L.wts);
    V.tsum = reinterpret_cast<float*>(at(ws, L.tsum));
    V.wq = P->t.resp ? reinterpret_cast<const float*>(at(ws, L.wq)) : nullptr;
    V.far_off = L.far_off;
    V.wt = wt;
    V.sino_stride = (long long)P->g.n_angles * P->g.n_bins;
    V.wts_stride = P->support;
    const long long n2 = (long long)P->g.n * P->g.n;
    V.gpart = reinterpret_cast<float*>(at(ws, L.gpart_cg));
    V.gpart_group_stride = 2 * n2;
    V.gpart_slice_stride = 0;
    V.tiles_x = P->tiles_x;
    set_groups(V, sh);
    {
        Timed t_(PGET_KC_VJP, stream);
        launch_vjp(P, V, 1, stream);
    }
    {
        Timed t_(PGET_KC_VECTOR, stream);
        hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, stream, (int)n2,
                           sh.n_part, sh.gfold, V.gpart, (long long)V.gpart_group_stride, gf, gmu);
    }
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

}  // extern "C"

// ------------------------------------------------------------------ solver
namespace {

// Range checks of the solver parameters (the ranges pget.h states).
bool params_ok(const pget_lm_params* p)
{
    if (!p) return false;
    if (p->max_outer < 1 || p->max_outer > 256 || p->n_cg < 1 || p->n_cg > 256) return false;
    if (!(p->alpha_f >= 0) || !(p->alpha_mu >= 0) || !(p->alpha_decay >= 1.0)) return false;
    if (!(p->d_f > 0) || !(p->d_mu > 0) || !(p->eta >= 0) || !(p->tau > 0)) return false;
    if (!(p->f_lo <= p->f_hi) || !(p->mu_lo <= p->mu_hi)) return false;
    if (!(p->tol >= 0)) return false;
    if (!(p->w_f >= 0) || !(p->w_mu >= 0) || !isfinite(p->w_f) || !isfinite(p->w_mu)) return false;
    if (p->active_set != 0 && p->active_set != 1) return false;
    if (p->step != PGET_STEP_CG && p->step != PGET_STEP_SGP) return false;
    return true;
}

// The per-slice parameters as the kernels read them.
LMParamsDev to_dev(const pget_lm_params& p)
{
    LMParamsDev d = {};
    d.alpha_f = p.alpha_f;
    d.alpha_mu = p.alpha_mu;
    d.alpha_decay = p.alpha_decay;
    d.alpha_decay_until = p.alpha_decay_until;
    d.max_outer = p.max_outer;
    d.n_cg = p.n_cg;
    d.beta0 = p.beta0;
    d.tau = p.tau;
    d.eta = p.eta;
    d.d_f = p.d_f;
    d.d_mu = p.d_mu;
    d.f_lo = p.f_lo;
    d.f_hi = p.f_hi;
    d.mu_lo = p.mu_lo;
    d.mu_hi = p.mu_hi;
    d.tol = p.tol;
    d.w_f = p.w_f > 0 ? p.w_f : 1.0;
    d.w_mu = p.w_mu > 0 ? p.w_mu : 1.0;
    d.active_set = p.active_set;
    d.prior_w = p.prior_w;
    d.prior_ref = p.prior_w ? p.prior_ref : nullptr;
    d.trace_u = p.trace_u;
    d.trace_t = p.trace_t;
    d.step_sgp = p.step == PGET_STEP_SGP ? 1 : 0;
    d.has_replay = p.replay != nullptr;
    if (p.replay)
        for (int k = 0; k < p.max_outer; ++k) d.replay[k] = p.replay[k];
    return d;
}

struct Solve {
    const pget_plan* P;
    int B;
    Shapes sh;
    Layout L;
    void* ws;
    hipStream_t stream;
    MarchArgs lin, trial;
    JvpArgs jcg, jsgp, jpred, jones;
    VjpArgs vgrad, vcg;
    VecArgs V;
    void* gimg;
};

// Argument blocks of every launch of a solve, pointing into its workspace:
// the linearising and trial marches, the Jacobian products (CG normal
// operator, ||J s||^2, ||J 1||^2), the two gathers (gradient and CG) and the
// vector kernels.
void setup(Solve& S)
{
    const pget_plan* P = S.P;
    const Geo& g = P->g;
    const long long n2 = (long long)g.n * g.n;
    const long long sino = (long long)g.n_angles * g.n_bins;
    const long long lat = P->support;   // compacted per-sample arrays
    void* ws = S.ws;
    double* part = reinterpret_cast<double*>(at(ws, S.L.part));
    float* u = reinterpret_cast<float*>(at(ws, S.L.u));
    float* ut = reinterpret_cast<float*>(at(ws, S.L.ut));
    LMState* st = reinterpret_cast<LMState*>(at(ws, S.L.state));
    void* wts = at(ws, S.L.wts);
    float* tsum = reinterpret_cast<float*>(at(ws, S.L.tsum));
    float* wq = P->t.resp ? reinterpret_cast<float*>(at(ws, S.L.wq)) : nullptr;
    float* wt_res = reinterpret_cast<float*>(at(ws, S.L.sino_a));   // K (A(u) - y)
    float* wt_cg = reinterpret_cast<float*>(at(ws, S.L.sino_b));    // K K J p
    const float* ymeas = reinterpret_cast<float*>(at(ws, S.L.ymeas));
    S.gimg = (P->lds_img && P->jvp_lds && P->jvp_bands == 1) ? nullptr : at(ws, S.L.gimg);

    MarchArgs& M = S.lin;
    M = MarchArgs{};
    M.g = g;
    M.t = P->t;
    M.src = planar_src(u, u + n2, 2 * n2);
    M.gimg = S.gimg;
    M.gimg_stride = (long long)g.pitch * g.pitch;
    M.wts = wts;
    M.tsum = tsum;
    M.wq = wq;
    M.far_off = S.L.far_off;
    M.wts_stride = lat;
    M.sino_stride = sino;
    M.ymeas = ymeas;
    M.wout = wt_res;
    M.part = part;
    M.slot = SLOT_PHI_DATA_U;
    M.st = st;
    M.angles_per_block = S.sh.apb;

    MarchArgs& T = S.trial;
    T = M;
    T.src = planar_src(ut, ut + n2, 2 * n2);
    T.wts = nullptr;
    T.tsum = nullptr;
    T.wq = nullptr;
    T.wout = nullptr;
    T.slot = SLOT_PHI_DATA_T;

    JvpArgs& J = S.jcg;
    J = JvpArgs{};
    J.g = g;
    J.t = P->t;
    J.gimg = S.gimg;
    J.gimg_stride = (long long)g.pitch * g.pitch;
    J.bands = P->jvp_bands;
    J.band_h = P->jvp_band_h;
    J.wts = wts;
    J.tsum = tsum;
    J.wq = wq;
    J.far_off = S.L.far_off;
    J.wts_stride = lat;
    J.sino_stride = sino;
    J.out = wt_cg;
    J.part = part;
    J.st = st;
    J.angles_per_block = S.sh.japb;
    float* r = reinterpret_cast<float*>(at(ws, S.L.r));
    float* p = reinterpret_cast<float*>(at(ws, S.L.p));
    J.src = PairSrc{};
    J.src.af = r;
    J.src.am = r + n2;
    J.src.bf = p;
    J.src.bm = p + n2;
    J.src.stride = 2 * n2;
    J.src.kind = 1;
    J.src.n_rr = S.sh.n_ew_blocks;
    J.src.prm = reinterpret_cast<const LMParamsDev*>(at(ws, S.L.params));

    // the scaled gradient projection's direction, formed by the vector kernels
    S.jsgp = J;
    S.jsgp.src = planar_src(p, p + n2, 2 * n2);

    float* s = reinterpret_cast<float*>(at(ws, S.L.s));
    S.jpred = J;
    S.jpred.src = planar_src(s, s + n2, 2 * n2);
    S.jpred.out = nullptr;
    S.jpred.slot = SLOT_JS;
    S.jones = S.jpred;
    S.jones.src.kind = 2;
    S.jones.slot = SLOT_J1;

    VjpArgs& VG = S.vgrad;
    VG = VjpArgs{};
    VG.g = g;
    VG.t = P->t;
    VG.wts = wts;
    VG.tsum = tsum;
    VG.wq = wq;
    VG.far_off = S.L.far_off;
    VG.wt = wt_res;
    VG.wts_stride = lat;
    VG.sino_stride = sino;
    VG.gpart = reinterpret_cast<float*>(at(ws, S.L.gpart_grad));
    VG.gpart_group_stride = (long long)S.B * 2 * n2;
    VG.gpart_slice_stride = 2 * n2;
    VG.tiles_x = P->tiles_x;
    set_groups(VG, S.sh);
    VG.st = st;
    VG.skip_if_clean = 1;
    S.vcg = VG;
    S.vcg.wt = wt_cg;
    S.vcg.gpart = reinterpret_cast<float*>(at(ws, S.L.gpart_cg));
    S.vcg.skip_if_clean = 0;

    VecArgs& V = S.V;
    V = VecArgs{};
    V.g = g;
    V.vstride = 2 * n2;
    V.u = u;
    V.ut = ut;
    V.s = s;
    V.x = reinterpret_cast<float*>(at(ws, S.L.x));
    V.r = r;
    V.p = p;
    V.q = reinterpret_cast<float*>(at(ws, S.L.q));
    V.grad = reinterpret_cast<float*>(at(ws, S.L.grad));
    V.fmask = reinterpret_cast<uint8_t*>(at(ws, S.L.fmask));
    V.gpart = S.vcg.gpart;
    V.gpart_group_stride = S.vcg.gpart_group_stride;
    V.gpart_slice_stride = S.vcg.gpart_slice_stride;
    V.groups = S.sh.n_part;
    V.gfold = S.sh.gfold;
    V.part = part;
    V.n_ew_blocks = S.sh.n_ew_blocks;
    V.n_angle_parts = g.n_angles;
    V.st = st;
    V.prm = reinterpret_cast<LMParamsDev*>(at(ws, S.L.params));
    V.rep = reinterpret_cast<ReportDev*>(at(ws, S.L.repdev));
}

// A ray march over every slice of the solve (through a bordered copy in HBM
// when the map pair does not fit in LDS).
void enqueue_march(Solve& S, const MarchArgs& A, int mode)
{
    if (!S.P->lds_img) pack(S.P, A.src, A.part, S.gimg, S.B, A.st, S.stream);
    if (mode == MARCH_LIN) march<MARCH_LIN>(S.P, A, S.sh.n_op_blocks, S.B, S.stream);
    else march<MARCH_TRIAL>(S.P, A, S.sh.n_op_blocks, S.B, S.stream);
}

// A Jacobian product over every slice of the solve (the same fallback).
void enqueue_jvp(Solve& S, const JvpArgs& A, int mode)
{
    if (S.sh.jvp_img == IMG_HBM) pack(S.P, A.src, A.part, S.gimg, S.B, A.st, S.stream, true);
    if (mode == JVP_NORMAL) jvp<JVP_NORMAL>(S.P, A, S.sh, S.B, S.stream);
    else jvp<JVP_SQNORM>(S.P, A, S.sh, S.B, S.stream);
}

// Model decrease and objective of the step held in ut (k_trial already run):
// ||J s||^2 and Phi(u').
void enqueue_step_eval(Solve& S)
{
    enqueue_jvp(S, S.jpred, JVP_SQNORM);
    enqueue_march(S, S.trial, MARCH_TRIAL);
}

// One outer LM iteration (Sec. 2.2): linearise at u (weights, Phi, the
// blurred residual); at k = 0 the initial damping unless given; the gradient
// g = J^T r + R u; n_cg CG steps on (J^T J + beta D + R) x = -g, each a
// product K^T K J p, a gather and the q / x updates; the trial point
// u' = clamp(u + x); the model decrease and Phi(u'); the decision (rho, beta).
// Every decision is taken on the device.
void enqueue_iteration(Solve& S, int k, int n_cg, bool need_beta0, bool hook_present, bool trace,
                       bool pool = false, bool sgp = false)
{
    const dim3 ew(S.sh.n_ew_blocks, S.B);
    enqueue_march(S, S.lin, MARCH_LIN);
    // the initial damping: at k = 0 of a solve, or in a slot pool (slots at
    // different iterations) for the slices at iteration 0
    if ((k == 0 && need_beta0) || pool) {
        JvpArgs J1 = S.jones;
        J1.only_k0 = pool ? 1 : 0;
        enqueue_jvp(S, J1, JVP_SQNORM);
        {
            Timed t_(PGET_KC_CONTROL, S.stream);
            hipLaunchKernelGGL(k_beta0, dim3(S.B), dim3(256), 0, S.stream, S.V);
        }
    }
    {
        Timed t_(PGET_KC_GRADIENT, S.stream);
        launch_vjp(S.P, S.vgrad, S.B, S.stream);
    }
    VecArgs Vg = S.V;
    Vg.gpart = S.vgrad.gpart;
    {
        Timed t_(PGET_KC_VECTOR, S.stream);
        hipLaunchKernelGGL(k_grad_init, ew, dim3(EW_THREADS), 0, S.stream, Vg);
    }
    for (int m = 0; m < n_cg && sgp; ++m) {
        // scaled gradient projection: M d, the step's line search and
        // steplength, the move and the next direction
        enqueue_jvp(S, S.jsgp, JVP_NORMAL);
        {
            Timed t_(PGET_KC_VJP, S.stream);
            launch_vjp(S.P, S.vcg, S.B, S.stream);
        }
        VecArgs V = S.V;
        V.cg_step = m;
        {
            Timed t_(PGET_KC_VECTOR, S.stream);
            hipLaunchKernelGGL(k_sgp_q, ew, dim3(EW_THREADS), 0, S.stream, V);
        }
        {
            Timed t_(PGET_KC_CONTROL, S.stream);
            hipLaunchKernelGGL(k_sgp_step, dim3(S.B), dim3(256), 0, S.stream, V);
        }
        {
            Timed t_(PGET_KC_VECTOR, S.stream);
            hipLaunchKernelGGL(k_sgp_x, ew, dim3(EW_THREADS), 0, S.stream, V);
        }
    }
    for (int m = 0; m < n_cg && !sgp; ++m) {
        JvpArgs J = S.jcg;
        J.src.rr_slot_cur = rr_slot(m);
        J.src.rr_slot_prev = rr_slot(m + 2);
        J.src.first = (m == 0);
        enqueue_jvp(S, J, JVP_NORMAL);
        {
            Timed t_(PGET_KC_VJP, S.stream);
            launch_vjp(S.P, S.vcg, S.B, S.stream);
        }
        VecArgs V = S.V;
        V.cg_step = m;
        {
            Timed t_(PGET_KC_VECTOR, S.stream);
            hipLaunchKernelGGL(k_cg_q, ew, dim3(EW_THREADS), 0, S.stream, V);
        }
        {
            Timed t_(PGET_KC_VECTOR, S.stream);
            hipLaunchKernelGGL(k_cg_x, ew, dim3(EW_THREADS), 0, S.stream, V);
        }
    }
    VecArgs Vt = S.V;
    Vt.cg_step = n_cg;
    {
        Timed t_(PGET_KC_VECTOR, S.stream);
        hipLaunchKernelGGL(k_trial, ew, dim3(EW_THREADS), 0, S.stream, Vt);
    }
    if (trace) {
        Timed t_(PGET_KC_VECTOR, S.stream);
        hipLaunchKernelGGL(k_trace, ew, dim3(EW_THREADS), 0, S.stream, S.V);
    }
    enqueue_step_eval(S);
    {
        Timed t_(PGET_KC_CONTROL, S.stream);
        hipLaunchKernelGGL(k_decide, dim3(S.B), dim3(256), 0, S.stream, S.V, hook_present ? 1 : 0);
    }
}

// Apply the iteration's decision: the trial point replaces u where it was
// accepted, and every slice's state advances.
void enqueue_commit(Solve& S)
{
    const dim3 ew(S.sh.n_ew_blocks, S.B);
    {
        Timed t_(PGET_KC_VECTOR, S.stream);
        hipLaunchKernelGGL(k_accept, ew, dim3(EW_THREADS), 0, S.stream, S.V);
    }
    {
        Timed t_(PGET_KC_CONTROL, S.stream);
        hipLaunchKernelGGL(k_commit, dim3((S.B + 63) / 64), dim3(64), 0, S.stream, S.V.st, S.V.prm, S.B);
    }
}

// The hook path of Alg. 2 for slice 0 (batch 1): host round trip per
// accepted step.
pget_status run_hook(Solve& S, pget_refine_fn hook, void* user)
{
    LMState st;
    if (hipMemcpyAsync(&st, S.V.st, sizeof(LMState), hipMemcpyDeviceToHost, S.stream) != hipSuccess ||
        hipStreamSynchronize(S.stream) != hipSuccess)
        return PGET_ERR_HIP;
    if (st.done || !st.accepted) return PGET_OK;
    const long long n2 = (long long)S.P->g.n * S.P->g.n;
    float* prop = S.V.q;   // free after the CG solve: holds the proposal u~
    int rc = hook(user, S.V.u, S.V.u + n2, S.V.s, S.V.s + n2, prop, prop + n2, S.stream);
    if (rc != 0) return PGET_OK;
    // evaluate the proposal: s~ = u~ - u, m(s~), Phi(u~)
    VecArgs Vh = S.V;
    Vh.ut = prop;
    Vh.hook_mode = 1;
    const dim3 ew(S.sh.n_ew_blocks, S.B);
    {
        Timed t_(PGET_KC_VECTOR, S.stream);
        hipLaunchKernelGGL(k_trial, ew, dim3(EW_THREADS), 0, S.stream, Vh);
    }
    enqueue_jvp(S, S.jpred, JVP_SQNORM);
    MarchArgs T = S.trial;
    T.src = planar_src(prop, prop + n2, 2 * n2);
    T.slot = SLOT_PHI_DATA_H;
    enqueue_march(S, T, MARCH_TRIAL);
    {
        Timed t_(PGET_KC_CONTROL, S.stream);
        hipLaunchKernelGGL(k_hook_decide, dim3(S.B), dim3(256), 0, S.stream, Vh);
    }
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

// The device report arrays of one slice into the caller's report (on `s`).
void copy_report(const ReportDev& R, const pget_lm_report* out, int max_outer, int n_cg, hipStream_t s)
{
    if (!out) return;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (dst) (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s);
    };
    cp(out->scalars, R.scalars, 4 * sizeof(double));
    cp(out->phi, R.phi, (size_t)(max_outer + 1) * sizeof(double));
    cp(out->rho, R.rho, (size_t)max_outer * sizeof(double));
    cp(out->beta, R.beta, (size_t)max_outer * sizeof(double));
    cp(out->pred, R.pred, (size_t)max_outer * sizeof(double));
    cp(out->ared, R.ared, (size_t)max_outer * sizeof(double));
    cp(out->gnorm, R.gnorm, (size_t)max_outer * sizeof(double));
    cp(out->accepted, R.accepted, (size_t)max_outer);
    cp(out->hook_accepted, R.hook_accepted, (size_t)max_outer);
    cp(out->cg_rr, R.cg_rr, (size_t)max_outer * n_cg * sizeof(double));
    cp(out->hook_rho, R.hook_rho, (size_t)max_outer * sizeof(double));
    cp(out->hook_pred, R.hook_pred, (size_t)max_outer * sizeof(double));
}

// One group of slices sharing a plan: its solve state and host-side copies
// of parameters and report descriptors.
struct Group {
    Solve S;
    int max_outer = 0, n_cg = 0;
    bool need_beta0 = false;
    bool trace = false;      // some slice records its iterates
    bool sgp = false;        // the step by scaled gradient projection (all slices)
    std::vector<LMParamsDev> prm;
    std::vector<ReportDev> rep;
    std::vector<const float*> y;
    std::vector<float*> f, mu;
    std::vector<const pget_lm_report*> reports;
};

// Internal streams (default priority) and events for fork/join.
struct StreamPool {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipStream_t get(size_t k)
    {
        while (streams.size() <= k) {
            hipStream_t s = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
            streams.push_back(s);
        }
        return streams[k];
    }
    hipEvent_t event(size_t k)
    {
        while (events.size() <= k) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
            events.push_back(e);
        }
        return events[k];
    }
} g_pool;


// Workspace of B slices of one plan (report arrays for the largest solve).
size_t group_bytes(const pget_plan* P, int B)
{
    Shapes sh = shapes_for(P, B);
    return align_up(layout_for(P, PGET_OP_LM, B, sh, 256, 256).total);
}

// Device report arrays of every slice of a solve, in its workspace.
void report_arrays(const Solve& S, int max_outer, int n_cg, std::vector<ReportDev>& rep)
{
    rep.assign(S.B, ReportDev{});
    const size_t per = align_up((size_t)(max_outer + 1) * 8 * sizeof(double) + 2 * (size_t)max_outer +
                                (size_t)max_outer * n_cg * sizeof(double) + 4 * sizeof(double) + 64);
    for (int b = 0; b < S.B; ++b) {
        char* base = at(S.ws, S.L.reparr + (size_t)b * per);
        size_t o = 0;
        auto take = [&](size_t bytes) { char* p = base + o; o += (bytes + 7) / 8 * 8; return p; };
        ReportDev& R = rep[b];
        R.phi = reinterpret_cast<double*>(take((max_outer + 1) * sizeof(double)));
        R.rho = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.beta = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.pred = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.ared = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.gnorm = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.cg_rr = reinterpret_cast<double*>(take((size_t)max_outer * n_cg * sizeof(double)));
        R.hook_rho = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.hook_pred = reinterpret_cast<double*>(take(max_outer * sizeof(double)));
        R.scalars = reinterpret_cast<double*>(take(4 * sizeof(double)));
        R.accepted = reinterpret_cast<int8_t*>(take(max_outer));
        R.hook_accepted = reinterpret_cast<int8_t*>(take(max_outer));
    }
}

// Validate, lay out and upload one group (uploads on `stream`).
pget_status group_prepare(Group& G, const pget_plan* P, int B, void* ws, hipStream_t stream)
{
    const pget_lm_params* params = nullptr;
    (void)params;
    G.max_outer = G.prm.empty() ? 0 : G.prm[0].max_outer;
    G.n_cg = G.prm.empty() ? 0 : G.prm[0].n_cg;
    G.need_beta0 = false;
    G.trace = false;
    G.sgp = !G.prm.empty() && G.prm[0].step_sgp;
    for (int b = 0; b < B; ++b) {
        if ((G.prm[b].step_sgp != 0) != G.sgp) return PGET_ERR_INVALID_ARG;
        if (G.prm[b].max_outer != G.max_outer || G.prm[b].n_cg != G.n_cg) return PGET_ERR_INVALID_ARG;
        if (!G.y[b] || !G.f[b] || !G.mu[b]) return PGET_ERR_INVALID_ARG;
        if (G.prm[b].beta0 <= 0.0) G.need_beta0 = true;
        if (G.prm[b].trace_u || G.prm[b].trace_t) G.trace = true;
    }
    Solve& S = G.S;
    S.P = P;
    S.B = B;
    S.sh = shapes_for(P, B);
    S.L = layout_for(P, PGET_OP_LM, B, S.sh, 256, 256);
    S.ws = ws;
    S.stream = stream;
    setup(S);
    const Geo& g = P->g;
    const size_t n2 = (size_t)g.n * g.n, sino = (size_t)g.n_angles * g.n_bins;
    const int max_outer = G.max_outer, n_cg = G.n_cg;
    report_arrays(S, max_outer, n_cg, G.rep);
    HIP_TRY(hipMemcpyAsync(const_cast<LMParamsDev*>(S.V.prm), G.prm.data(), B * sizeof(LMParamsDev),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(S.V.rep, G.rep.data(), B * sizeof(ReportDev), hipMemcpyHostToDevice, stream));
    float* ymeas = reinterpret_cast<float*>(at(ws, S.L.ymeas));
    for (int b = 0; b < B; ++b) {
        HIP_TRY(hipMemcpyAsync(ymeas + b * sino, G.y[b], sino * sizeof(float), hipMemcpyDeviceToDevice, stream));
        HIP_TRY(hipMemcpyAsync(S.V.u + b * 2 * n2, G.f[b], n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
        HIP_TRY(hipMemcpyAsync(S.V.u + b * 2 * n2 + n2, G.mu[b], n2 * sizeof(float), hipMemcpyDeviceToDevice,
                               stream));
    }
    return PGET_OK;
}

// The whole device-resident solve of one group (no hook).
void group_begin(Group& G, hipStream_t s)
{
    const int B = G.S.B;
    hipLaunchKernelGGL(k_lm_init, dim3((B + 63) / 64), dim3(64), 0, s, G.S.V.st, G.S.V.prm, B);
}

void group_iteration(Group& G, hipStream_t s, int k)
{
    Solve SS = G.S;
    SS.stream = s;
    enqueue_iteration(SS, k, G.n_cg, G.need_beta0, false, G.trace, false, G.sgp);
    enqueue_commit(SS);
}

void group_end(Group& G, hipStream_t s)
{
    const int B = G.S.B;
    hipLaunchKernelGGL(k_final_reg, dim3(G.S.sh.n_ew_blocks, B), dim3(EW_THREADS), 0, s, G.S.V);
    hipLaunchKernelGGL(k_finish, dim3(B), dim3(256), 0, s, G.S.V);
}

void enqueue_group(Group& G, hipStream_t s)
{
    group_begin(G, s);
    for (int k = 0; k < G.max_outer; ++k) group_iteration(G, s, k);
    group_end(G, s);
}

// All groups forked from `origin` onto their own streams and joined back.
// The groups' launches are enqueued interleaved, one outer iteration of
// every group in turn: a captured graph keeps that order, so every group
// starts at once instead of each waiting until the launches of the groups
// before it have been submitted.
pget_status enqueue_forked(std::vector<Group>& groups, hipStream_t origin, size_t stream_base)
{
    if (groups.size() == 1) {
        enqueue_group(groups[0], origin);
        return PGET_OK;
    }
    hipEvent_t fork = g_pool.event(0);
    if (!fork) return PGET_ERR_HIP;
    HIP_TRY(hipEventRecord(fork, origin));
    std::vector<hipStream_t> st(groups.size());
    int kmax = 0;
    for (size_t k = 0; k < groups.size(); ++k) {
        st[k] = g_pool.get(stream_base + k);
        if (!st[k]) return PGET_ERR_HIP;
        HIP_TRY(hipStreamWaitEvent(st[k], fork, 0));
        group_begin(groups[k], st[k]);
        kmax = std::max(kmax, groups[k].max_outer);
    }
    for (int it = 0; it < kmax; ++it)
        for (size_t k = 0; k < groups.size(); ++k)
            if (it < groups[k].max_outer) group_iteration(groups[k], st[k], it);
    for (size_t k = 0; k < groups.size(); ++k) {
        group_end(groups[k], st[k]);
        hipEvent_t done = g_pool.event(1 + k);
        if (!done) return PGET_ERR_HIP;
        HIP_TRY(hipEventRecord(done, st[k]));
        HIP_TRY(hipStreamWaitEvent(origin, done, 0));
    }
    return PGET_OK;
}

pget_status solve_groups(std::vector<Group>& groups, pget_refine_fn hook, void* hook_user, void* ws,
                         hipStream_t stream)
{
    // uploads went through host vectors owned by `groups`; wait for them
    HIP_TRY(hipStreamSynchronize(stream));
    const bool graph_ok = g_use_graphs && !hook && g_timing.classes == 0;
    if (hook) {
        Group& G = groups[0];
        Solve& S = G.S;
        const int B = S.B;
        hipLaunchKernelGGL(k_lm_init, dim3((B + 63) / 64), dim3(64), 0, stream, S.V.st, S.V.prm, B);
        for (int k = 0; k < G.max_outer; ++k) {
            enqueue_iteration(S, k, G.n_cg, G.need_beta0, true, G.trace, false, G.sgp);
            pget_status rc = run_hook(S, hook, hook_user);
            if (rc != PGET_OK) return rc;
            enqueue_commit(S);
        }
        hipLaunchKernelGGL(k_final_reg, dim3(S.sh.n_ew_blocks, B), dim3(EW_THREADS), 0, stream, S.V);
        hipLaunchKernelGGL(k_finish, dim3(B), dim3(256), 0, stream, S.V);
    } else if (!graph_ok) {
        pget_status rc = enqueue_forked(groups, stream, 1);
        if (rc != PGET_OK) return rc;
    } else {
        GraphKey key;
        key.ws = ws;
        for (auto& G : groups)
            key.groups.push_back({(long long)(intptr_t)G.S.P, G.S.B, G.max_outer, G.n_cg,
                                  (long long)G.need_beta0 | ((long long)G.trace << 1) | ((long long)G.sgp << 2),
                                  (long long)((char*)G.S.ws - (char*)ws)});
        hipGraphExec_t exec = nullptr;
        ++g_graph_clock;
        for (auto& e : g_graphs)
            if (e.key == key) {
                exec = e.exec;
                e.used = g_graph_clock;
            }
        if (!exec) {
            if (g_graphs.size() >= GRAPH_CACHE) {
                // earlier replays of the evicted graph may still run on
                // some stream: wait for the device before destroying it
                HIP_TRY(hipDeviceSynchronize());
                size_t lru = 0;
                for (size_t k = 1; k < g_graphs.size(); ++k)
                    if (g_graphs[k].used < g_graphs[lru].used) lru = k;
                (void)hipGraphExecDestroy(g_graphs[lru].exec);
                g_graphs.erase(g_graphs.begin() + lru);
            }
            hipStream_t cs = g_pool.get(0);
            if (!cs) return PGET_ERR_HIP;
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            pget_status rc = enqueue_forked(groups, cs, 1);
            hipError_t ee = hipStreamEndCapture(cs, &graph);
            if (rc != PGET_OK) return rc;
            if (ee != hipSuccess) return PGET_ERR_HIP;
            hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return PGET_ERR_HIP;
            g_graphs.push_back(GraphEntry{key, exec, g_graph_clock});
        }
        HIP_TRY(hipGraphLaunch(exec, stream));
    }
    for (auto& G : groups) {
        const Geo& g = G.S.P->g;
        const size_t n2 = (size_t)g.n * g.n;
        for (int b = 0; b < G.S.B; ++b) {
            HIP_TRY(hipMemcpyAsync(G.f[b], G.S.V.u + b * 2 * n2, n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
            HIP_TRY(hipMemcpyAsync(G.mu[b], G.S.V.u + b * 2 * n2 + n2, n2 * sizeof(float),
                                   hipMemcpyDeviceToDevice, stream));
            if (G.reports[b]) copy_report(G.rep[b], G.reports[b], G.max_outer, G.n_cg, stream);
        }
    }
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

// B slices of one plan in the same launches.
pget_status solve_impl(const pget_plan* P, int B, const float* const* y, float* const* f,
                       float* const* mu, const pget_lm_params* params, const pget_lm_report* reports,
                       pget_refine_fn hook, void* hook_user, void* ws, hipStream_t stream)
{
    if (!P || B < 1 || !y || !f || !mu || !params) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    if (hook && B != 1) return PGET_ERR_INVALID_ARG;
    std::vector<Group> groups(1);
    Group& G = groups[0];
    for (int b = 0; b < B; ++b) {
        if (!params_ok(&params[b])) return PGET_ERR_INVALID_ARG;
        G.prm.push_back(to_dev(params[b]));
        G.y.push_back(y[b]);
        G.f.push_back(f[b]);
        G.mu.push_back(mu[b]);
        G.reports.push_back(reports ? &reports[b] : nullptr);
    }
    pget_status rc = group_prepare(G, P, B, ws, stream);
    if (rc != PGET_OK) return rc;
    return solve_groups(groups, hook, hook_user, ws, stream);
}

// Slices of several plans: one group per plan, on forked streams.
pget_status solve_multi(int n, const pget_plan* const* plans, const float* const* y, float* const* f,
                        float* const* mu, const pget_lm_params* params, const pget_lm_report* reports,
                        void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (n < 1 || !plans || !y || !f || !mu || !params) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    // groups by plan, in order of first appearance
    std::vector<const pget_plan*> order;
    std::vector<std::vector<int>> members;
    for (int s = 0; s < n; ++s) {
        if (!plans[s] || !params_ok(&params[s])) return PGET_ERR_INVALID_ARG;
        size_t k = 0;
        while (k < order.size() && order[k] != plans[s]) ++k;
        if (k == order.size()) {
            order.push_back(plans[s]);
            members.emplace_back();
        }
        members[k].push_back(s);
    }
    std::vector<Group> groups(order.size());
    size_t off = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const int B = (int)members[k].size();
        const size_t bytes = group_bytes(order[k], B);
        if (off + bytes > ws_bytes) return PGET_ERR_WORKSPACE;
        Group& G = groups[k];
        for (int s : members[k]) {
            G.prm.push_back(to_dev(params[s]));
            G.y.push_back(y[s]);
            G.f.push_back(f[s]);
            G.mu.push_back(mu[s]);
            G.reports.push_back(reports ? &reports[s] : nullptr);
        }
        pget_status rc = group_prepare(G, order[k], B, at(ws, off), stream);
        if (rc != PGET_OK) return rc;
        off += bytes;
    }
    return solve_groups(groups, nullptr, nullptr, ws, stream);
}

}  // namespace

extern "C" {

pget_status pget_set_graphs(int32_t enable)
{
    g_use_graphs = enable != 0;
    return PGET_OK;
}

pget_status pget_timing_enable(int32_t classes, int32_t capacity)
{
    if (capacity < 0) return PGET_ERR_INVALID_ARG;
    for (hipEvent_t e : g_timing.pool) (void)hipEventDestroy(e);
    g_timing.pool.clear();
    g_timing.recs.clear();
    g_timing.classes = 0;
    g_timing.capacity = 0;
    if (capacity == 0 || classes == 0) return PGET_OK;
    g_timing.pool.resize(2 * (size_t)capacity);
    for (auto& e : g_timing.pool)
        if (hipEventCreate(&e) != hipSuccess) return PGET_ERR_HIP;
    g_timing.recs.reserve(capacity);
    g_timing.classes = classes;
    g_timing.capacity = capacity;
    return PGET_OK;
}

pget_status pget_timing_read(int32_t kernel_class, double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return PGET_ERR_INVALID_ARG;
    double sum = 0.0;
    int64_t cnt = 0;
    for (const TimingRec& r : g_timing.recs) {
        if (r.cls != kernel_class) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return PGET_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return PGET_ERR_HIP;
        sum += ms;
        ++cnt;
    }
    *total_ms = sum;
    *launches = cnt;
    return PGET_OK;
}

pget_status pget_lm_solve(const pget_plan* plan, const float* y, float* f_inout, float* mu_inout,
                          const pget_lm_params* params, pget_refine_fn hook, void* hook_user,
                          const pget_lm_report* report, void* ws, hipStream_t stream)
{
    const float* ys[1] = {y};
    float* fs[1] = {f_inout};
    float* ms[1] = {mu_inout};
    return solve_impl(plan, 1, ys, fs, ms, params, report, hook, hook_user, ws, stream);
}

pget_status pget_autotune(pget_plan* P, int32_t batch, void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (!P || batch < 1) return PGET_ERR_INVALID_ARG;
    if (!ws || ws_bytes < group_bytes(P, batch)) return PGET_ERR_WORKSPACE;
    // captured solver sequences of this plan used the old shapes
    drop_graphs(P);
    // drop an earlier choice for this batch so that the candidates below rule
    for (size_t k = 0; k < P->tuned.size(); ++k)
        if (P->tuned[k][0] == batch) {
            P->tuned.erase(P->tuned.begin() + k);
            break;
        }
    fill_zero(ws, group_bytes(P, batch), stream);
    const int slots = P->g.paired ? P->g.n_angles / 2 : P->g.n_angles;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto time_it = [&](auto&& launch) -> float {
        launch();   // warm
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, stream);
            launch();
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    int best_japb = 1, best_groups = 1;
    float best_j = 1e30f, best_v = 1e30f;
    // candidates share one workspace layout: the layout only depends on the
    // largest group count, so size the search within what the workspace holds
    Solve S;
    S.P = P;
    S.B = batch;
    S.sh = shapes_for(P, batch);
    S.L = layout_for(P, PGET_OP_LM, batch, S.sh, 256, 256);
    S.ws = ws;
    S.stream = stream;
    setup(S);
    for (int japb = 1; japb <= max_japb_of(P); japb *= 2) {
        Shapes sh = S.sh;
        set_japb(P, sh, japb);
        JvpArgs J = S.jcg;
        J.src = planar_src(S.V.u, S.V.u + (size_t)P->g.n * P->g.n, 2LL * P->g.n * P->g.n);
        J.st = nullptr;
        J.angles_per_block = japb;
        const float t = time_it([&] {
            if (sh.jvp_img == IMG_HBM) pack(P, J.src, nullptr, S.gimg, batch, nullptr, stream, true);
            jvp<JVP_NORMAL>(P, J, sh, batch, stream);
        });
        if (t < best_j) { best_j = t; best_japb = japb; }
    }
    // the partial-image buffers hold the fine groups, the most any layout writes
    for (int fpb : fpb_candidates(S.sh.fine, S.sh.gs)) {
        Shapes sh = S.sh;
        set_fpb(sh, fpb);
        VjpArgs V = S.vcg;
        V.st = nullptr;
        set_groups(V, sh);
        const float t = time_it([&] {
            launch_vjp(P, V, batch, stream);
        });
        if (t < best_v) { best_v = t; best_groups = sh.fpb; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->tuned.push_back({batch, best_japb, best_groups});
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

pget_status pget_set_shape(pget_plan* P, int32_t batch, int32_t japb, int32_t fine_per_block)
{
    if (!P || batch < 1 || japb < 0 || fine_per_block < 0) return PGET_ERR_INVALID_ARG;
    if (japb > max_japb_of(P)) return PGET_ERR_INVALID_ARG;
    const Shapes def = shapes_for(P, batch);
    // captured solver sequences of this plan used the old shapes
    drop_graphs(P);
    for (size_t k = 0; k < P->tuned.size(); ++k)
        if (P->tuned[k][0] == batch) {
            P->tuned.erase(P->tuned.begin() + k);
            break;
        }
    P->tuned.push_back({batch, japb > 0 ? japb : def.japb, fine_per_block > 0 ? fine_per_block : def.fpb});
    return PGET_OK;
}

int32_t pget_tuned_shape(const pget_plan* P, int32_t batch, int32_t* japb, int32_t* vjp_groups)
{
    if (!P || batch < 1) return 0;
    Shapes sh = shapes_for(P, batch);
    if (japb) *japb = sh.japb;
    if (vjp_groups) *vjp_groups = sh.groups;
    for (const auto& t : P->tuned)
        if (t[0] == batch) return 1;
    return 0;
}

size_t pget_workspace_bytes_multi(int32_t n_slices, const pget_plan* const* plans)
{
    if (n_slices < 1 || !plans) return 0;
    std::vector<const pget_plan*> order;
    std::vector<int> counts;
    for (int s = 0; s < n_slices; ++s) {
        if (!plans[s]) return 0;
        size_t k = 0;
        while (k < order.size() && order[k] != plans[s]) ++k;
        if (k == order.size()) {
            order.push_back(plans[s]);
            counts.push_back(0);
        }
        ++counts[k];
    }
    size_t total = 0;
    for (size_t k = 0; k < order.size(); ++k) total += group_bytes(order[k], counts[k]);
    return total;
}

pget_status pget_lm_solve_multi(int32_t n_slices, const pget_plan* const* plans, const float* const* y,
                                float* const* f_inout, float* const* mu_inout,
                                const pget_lm_params* params, const pget_lm_report* reports, void* ws,
                                size_t ws_bytes, hipStream_t stream)
{
    return solve_multi(n_slices, plans, y, f_inout, mu_inout, params, reports, ws, ws_bytes, stream);
}

pget_status pget_lm_solve_batched(const pget_plan* plan, int32_t n_slices, const float* const* y,
                                  float* const* f_inout, float* const* mu_inout,
                                  const pget_lm_params* params, const pget_lm_report* reports,
                                  void* ws, hipStream_t stream)
{
    return solve_impl(plan, n_slices, y, f_inout, mu_inout, params, reports, nullptr, nullptr, ws, stream);
}

}  // extern "C"

// ------------------------------------------------------------ slot pools
// Continuous batching at outer-iteration boundaries: `cap` slots of one
// plan share every launch of an outer iteration; each slot holds one
// slice's whole LM state on the device and runs at its own iteration count.
struct pget_lm_pool {
    const pget_plan* P = nullptr;
    int cap = 0, max_outer = 0, n_cg = 0;
    int step = PGET_STEP_CG;        // the damped step's solver of every slot
    Solve S;
    std::vector<LMParamsDev> prm;   // host copies of the slots' parameters
    std::vector<ReportDev> rep;     // the slots' device report arrays
    std::vector<char> loaded;       // host view: slot holds a slice
    int* flags = nullptr;           // device: 1 where a slot's solve has finished
    hipGraphExec_t step_graph = nullptr;
};

namespace {

size_t pool_bytes(const pget_plan* P, int cap, int max_outer, int n_cg, Layout* out)
{
    Shapes sh = shapes_for(P, cap);
    Layout L = layout_for(P, PGET_OP_LM, cap, sh, max_outer, n_cg);
    if (out) *out = L;
    return L.total + align_up((size_t)cap * sizeof(int));
}

// One outer iteration of every unfinished slot, then the report's objective
// and scalars of every slot and the finished flags.
void enqueue_pool_step(pget_lm_pool* Q, hipStream_t s)
{
    Solve S = Q->S;
    S.stream = s;
    enqueue_iteration(S, 1, Q->n_cg, true, false, true, true, Q->step == PGET_STEP_SGP);
    enqueue_commit(S);
    hipLaunchKernelGGL(k_final_reg, dim3(S.sh.n_ew_blocks, S.B), dim3(EW_THREADS), 0, s, S.V);
    hipLaunchKernelGGL(k_finish, dim3(S.B), dim3(256), 0, s, S.V);
    hipLaunchKernelGGL(k_pool_flags, dim3((S.B + 63) / 64), dim3(64), 0, s, S.V.st, Q->flags, S.B);
}

}  // namespace

extern "C" {

size_t pget_lm_pool_workspace_bytes(const pget_plan* plan, int32_t capacity, int32_t max_outer, int32_t n_cg)
{
    if (!plan || capacity < 1 || max_outer < 1 || max_outer > 256 || n_cg < 1 || n_cg > 256) return 0;
    return pool_bytes(plan, capacity, max_outer, n_cg, nullptr);
}

pget_status pget_lm_pool_create(const pget_plan* plan, int32_t capacity, int32_t max_outer, int32_t n_cg, int32_t step,
                                void* ws, size_t ws_bytes, hipStream_t stream, pget_lm_pool** out)
{
    if (!out) return PGET_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plan || capacity < 1 || max_outer < 1 || max_outer > 256 || n_cg < 1 || n_cg > 256)
        return PGET_ERR_INVALID_ARG;
    if (step != PGET_STEP_CG && step != PGET_STEP_SGP) return PGET_ERR_INVALID_ARG;
    if (!ws) return PGET_ERR_WORKSPACE;
    Layout L;
    const size_t need = pool_bytes(plan, capacity, max_outer, n_cg, &L);
    if (ws_bytes < need) return PGET_ERR_WORKSPACE;
    pget_lm_pool* Q = new (std::nothrow) pget_lm_pool();
    if (!Q) return PGET_ERR_HIP;
    Q->P = plan;
    Q->cap = capacity;
    Q->max_outer = max_outer;
    Q->n_cg = n_cg;
    Q->step = step;
    Solve& S = Q->S;
    S.P = plan;
    S.B = capacity;
    S.sh = shapes_for(plan, capacity);
    S.L = L;
    S.ws = ws;
    S.stream = stream;
    setup(S);
    Q->flags = reinterpret_cast<int*>(at(ws, L.total));
    Q->prm.assign(capacity, LMParamsDev{});
    Q->loaded.assign(capacity, 0);
    report_arrays(S, max_outer, n_cg, Q->rep);
    // every slot starts free (finished), with zeroed parameters: the report
    // kernels of a step (k_final_reg reads a slot's prior pointers) also run
    // over free slots
    bool ok = hipMemcpyAsync(const_cast<LMParamsDev*>(S.V.prm), Q->prm.data(), capacity * sizeof(LMParamsDev),
                             hipMemcpyHostToDevice, stream) == hipSuccess;
    hipLaunchKernelGGL(k_pool_clear, dim3((capacity + 63) / 64), dim3(64), 0, stream, S.V.st, capacity);
    hipLaunchKernelGGL(k_pool_flags, dim3((capacity + 63) / 64), dim3(64), 0, stream, S.V.st, Q->flags, capacity);
    ok = ok && hipMemcpyAsync(S.V.rep, Q->rep.data(), capacity * sizeof(ReportDev), hipMemcpyHostToDevice, stream) ==
                  hipSuccess &&
              hipStreamSynchronize(stream) == hipSuccess && hipGetLastError() == hipSuccess;
    if (!ok) {
        delete Q;
        return PGET_ERR_HIP;
    }
    *out = Q;
    return PGET_OK;
}

void pget_lm_pool_destroy(pget_lm_pool* pool)
{
    if (!pool) return;
    if (pool->step_graph) (void)hipGraphExecDestroy(pool->step_graph);
    delete pool;
}

pget_status pget_lm_pool_load(pget_lm_pool* Q, int32_t slot, const float* y, const float* f0, const float* mu0,
                              const pget_lm_params* params, hipStream_t stream)
{
    if (!Q || slot < 0 || slot >= Q->cap || !y || !f0 || !mu0 || !params_ok(params)) return PGET_ERR_INVALID_ARG;
    if (Q->loaded[slot] || params->max_outer > Q->max_outer || params->n_cg != Q->n_cg || params->step != Q->step)
        return PGET_ERR_INVALID_ARG;
    Solve& S = Q->S;
    const Geo& g = Q->P->g;
    const size_t n2 = (size_t)g.n * g.n, sino = (size_t)g.n_angles * g.n_bins;
    Q->prm[slot] = to_dev(*params);
    LMParamsDev* prm_dev = const_cast<LMParamsDev*>(S.V.prm) + slot;
    float* ymeas = reinterpret_cast<float*>(at(S.ws, S.L.ymeas));
    HIP_TRY(hipMemcpyAsync(prm_dev, &Q->prm[slot], sizeof(LMParamsDev), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ymeas + slot * sino, y, sino * sizeof(float), hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(S.V.u + slot * 2 * n2, f0, n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(S.V.u + slot * 2 * n2 + n2, mu0, n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_lm_init, dim3(1), dim3(64), 0, stream, S.V.st + slot, prm_dev, 1);
    HIP_TRY(hipGetLastError());
    Q->loaded[slot] = 1;
    return PGET_OK;
}

pget_status pget_lm_pool_step(pget_lm_pool* Q, int32_t* finished, hipStream_t stream)
{
    if (!Q) return PGET_ERR_INVALID_ARG;
    const bool graph_ok = g_use_graphs && g_timing.classes == 0;
    if (!graph_ok) {
        enqueue_pool_step(Q, stream);
    } else {
        if (!Q->step_graph) {
            hipStream_t cs = g_pool.get(0);
            if (!cs) return PGET_ERR_HIP;
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            enqueue_pool_step(Q, cs);
            HIP_TRY(hipStreamEndCapture(cs, &graph));
            hipError_t e = hipGraphInstantiate(&Q->step_graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                Q->step_graph = nullptr;
                return PGET_ERR_HIP;
            }
        }
        HIP_TRY(hipGraphLaunch(Q->step_graph, stream));
    }
    if (finished)
        HIP_TRY(hipMemcpyAsync(finished, Q->flags, Q->cap * sizeof(int), hipMemcpyDefault, stream));
    return hipGetLastError() == hipSuccess ? PGET_OK : PGET_ERR_HIP;
}

pget_status pget_lm_pool_fetch(pget_lm_pool* Q, int32_t slot, float* f_out, float* mu_out,
                               const pget_lm_report* report, hipStream_t stream)
{
    if (!Q || slot < 0 || slot >= Q->cap || !Q->loaded[slot]) return PGET_ERR_INVALID_ARG;
    Solve& S = Q->S;
    const size_t n2 = (size_t)Q->P->g.n * Q->P->g.n;
    if (f_out) HIP_TRY(hipMemcpyAsync(f_out, S.V.u + slot * 2 * n2, n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
    if (mu_out)
        HIP_TRY(hipMemcpyAsync(mu_out, S.V.u + slot * 2 * n2 + n2, n2 * sizeof(float), hipMemcpyDeviceToDevice, stream));
    if (report) copy_report(Q->rep[slot], report, Q->prm[slot].max_outer, Q->n_cg, stream);
    hipLaunchKernelGGL(k_pool_release, dim3(1), dim3(64), 0, stream, S.V.st, slot);
    HIP_TRY(hipGetLastError());
    // zeroed parameters: the freed slot's prior and trace pointers belong to
    // the caller and may not outlive the fetch
    Q->prm[slot] = LMParamsDev{};
    HIP_TRY(hipMemcpyAsync(const_cast<LMParamsDev*>(S.V.prm) + slot, &Q->prm[slot], sizeof(LMParamsDev),
                           hipMemcpyHostToDevice, stream));
    Q->loaded[slot] = 0;
    return PGET_OK;
}

}  // extern "C"
