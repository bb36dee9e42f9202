// Host side of the C ABI declared in include/cadmm.h: descriptor validation,
// workspace planning inside caller-owned device memory, work lists, HIP-graph
// capture of one ADMM iteration, launch-shape autotuning and result readout.
#include "cadmm.h"
#include "cadmm_internal.h"
#include "cadmm_model.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace cadmm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(CADMM_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr int kHistCap = 4096;
constexpr int kGraphBlock = 8;    // iterations per captured multi-iteration graph
constexpr int kPreSumWorkgroups = 128;   // workgroups per scenario from which the sums get their own kernel
constexpr int kTuneWarmIters = 16; // iterations run before the launch shapes are timed

struct Layout {
    // sizes
    int dim, n_s, n_u, N, n_parts, n_scen, M, Fr, Fo, n_blocks;
    long long n_pairs, y_floats;
    int nc, nq, n_att, max_pf, max_of;
    // byte offsets into the workspace
    size_t part_faces, part_face_ptr, part_off, obs_faces, obs_d64, obs_dc, obs_face_ptr, blocks, block_yoff, bdesc, wg_items,
        scen_wg;
    size_t A_dyn, B_dyn, c_dyn, Q_s, Q_u, x_ref, x0, A_lin, B_lin;
    long long n_models;
    size_t x, u, y, zeta, xi, y_snap, x_snap, u_snap;
    size_t contrib, rdual_part, rpri_part, unconv_part;
    size_t r_pri, r_dual, done, iters, unconv, hist_pri, hist_dual, alpha, cost, min_alpha;
    int has_bounds;
    size_t blim, hq_b, bW, bstat, bprev, hq_pre;
    size_t total;
};

size_t take(size_t& off, size_t bytes)
{
    off = (off + 255) & ~size_t(255);
    size_t r = off;
    off += bytes;
    return r;
}

bool finite_all(const double* p, long long n)
{
    if (n > 0 && !p) return false;
    for (long long i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int validate_and_plan(const cadmm_desc* d, Layout& L)
{
    if (!d) return fail(CADMM_INVALID, "descriptor is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(CADMM_INVALID, "dim must be 2 or 3");
    if (d->n_s < 1 || d->n_s > CADMM_MAX_NS) return fail(CADMM_INVALID, "n_s out of range");
    if (d->n_u < 1 || d->n_u > CADMM_MAX_NU) return fail(CADMM_INVALID, "n_u out of range");
    if (d->N < 1 || d->N > CADMM_MAX_N) return fail(CADMM_INVALID, "horizon N out of range (1..64)");
    if (d->n_parts < 1 || d->n_scen < 1) return fail(CADMM_INVALID, "need >= 1 robot part and scenario");
    if (d->n_parts > 32767) return fail(CADMM_INVALID, "more than 32767 robot parts");
    if (!d->part_face_ptr || !d->obs_ptr || !d->obs_face_ptr || !d->pos_idx || !d->att_idx)
        return fail(CADMM_INVALID, "NULL index array");
    const int dim = d->dim;
    const int want_att = dim == 2 ? CADMM_ATT_YAW : CADMM_ATT_EULER_ZYX;
    if (d->att_kind != want_att) return fail(CADMM_INVALID, "att_kind must be YAW for dim 2 and EULER_ZYX for dim 3");
    const int n_att = dim == 2 ? 1 : 3;
    for (int r = 0; r < dim; ++r)
        if (d->pos_idx[r] < 0 || d->pos_idx[r] >= d->n_s) return fail(CADMM_INVALID, "pos_idx out of range");
    for (int a = 0; a < n_att; ++a)
        if (d->att_idx[a] < 0 || d->att_idx[a] >= d->n_s) return fail(CADMM_INVALID, "att_idx out of range");
    if (d->part_face_ptr[0] != 0) return fail(CADMM_INVALID, "part_face_ptr[0] != 0");
    int max_pf = 0;
    for (int i = 0; i < d->n_parts; ++i) {
        const int nf = d->part_face_ptr[i + 1] - d->part_face_ptr[i];
        if (nf < dim + 1 || nf > CADMM_MAX_PART_FACES) return fail(CADMM_INVALID, "faces per robot part out of range");
        max_pf = std::max(max_pf, nf);
    }
    const int Fr = d->part_face_ptr[d->n_parts];
    if (!finite_all(d->part_A, (long long)Fr * dim) || !finite_all(d->part_b, Fr) ||
        !finite_all(d->part_off, (long long)d->n_parts * dim))
        return fail(CADMM_INVALID, "non-finite robot geometry");
    for (int k = 0; k < Fr; ++k) {
        if (!(d->part_b[k] > 0.0)) return fail(CADMM_INVALID, "robot offsets b_i must be > 0 (centre inside the part)");
        double nn = 0;
        for (int r = 0; r < dim; ++r) nn += d->part_A[k * dim + r] * d->part_A[k * dim + r];
        if (!(nn > 0.0)) return fail(CADMM_INVALID, "zero-norm robot face");
    }
    if (d->obs_ptr[0] != 0) return fail(CADMM_INVALID, "obs_ptr[0] != 0");
    for (int s = 0; s < d->n_scen; ++s)
        if (d->obs_ptr[s + 1] < d->obs_ptr[s]) return fail(CADMM_INVALID, "obs_ptr not monotone");
    const int M = d->obs_ptr[d->n_scen];
    if (d->obs_face_ptr[0] != 0) return fail(CADMM_INVALID, "obs_face_ptr[0] != 0");
    int max_of = 0;
    for (int j = 0; j < M; ++j) {
        const int nf = d->obs_face_ptr[j + 1] - d->obs_face_ptr[j];
        if (nf < dim + 1 || nf > CADMM_MAX_OBS_FACES) return fail(CADMM_INVALID, "faces per obstacle out of range");
        max_of = std::max(max_of, nf);
    }
    const int Fo = M > 0 ? d->obs_face_ptr[M] : 0;
    if (!finite_all(d->obs_C, (long long)Fo * dim) || !finite_all(d->obs_d, Fo))
        return fail(CADMM_INVALID, "non-finite obstacle geometry");
    for (int k = 0; k < Fo; ++k) {
        double nn = 0;
        for (int r = 0; r < dim; ++r) nn += d->obs_C[k * dim + r] * d->obs_C[k * dim + r];
        if (!(nn > 0.0)) return fail(CADMM_INVALID, "zero-norm obstacle face");
    }
    const int ns = d->n_s, nu = d->n_u, N = d->N;
    if (d->dyn_t_stride < 0 || d->dyn_s_stride < 0 || d->dyn_t_stride > (1 << 20) || d->dyn_s_stride > (1 << 20))
        return fail(CADMM_INVALID, "dynamics model strides out of range");
    const long long n_models = (long long)(d->n_scen - 1) * d->dyn_s_stride + (long long)(N - 1) * d->dyn_t_stride + 1;
    if (n_models * ns * ns >= (1LL << 31)) return fail(CADMM_INVALID, "too many dynamics models");
    if (d->model == CADMM_MODEL_BICYCLE) {
        if (dim != 2 || ns != 4 || nu != 2) return fail(CADMM_INVALID, "the bicycle model needs dim 2, n_s 4, n_u 2");
        if (!(d->model_par[0] > 0) || !(d->model_par[1] > 0) || !std::isfinite(d->model_par[0]) ||
            !std::isfinite(d->model_par[1]))
            return fail(CADMM_INVALID, "bicycle model_par: dt and wheelbase must be finite and > 0");
    } else if (d->model == CADMM_MODEL_QUADROTOR) {
        if (dim != 3 || ns != 12 || nu != 4) return fail(CADMM_INVALID, "the quadrotor model needs dim 3, n_s 12, n_u 4");
        for (int k = 0; k < 5; ++k)
            if (!(d->model_par[k] > 0) || !std::isfinite(d->model_par[k]))
                return fail(CADMM_INVALID, "quadrotor model_par: dt, mass and inertias must be finite and > 0");
        if (!std::isfinite(d->model_par[5])) return fail(CADMM_INVALID, "quadrotor model_par: g must be finite");
    } else if (d->model != CADMM_MODEL_LINEAR) {
        return fail(CADMM_INVALID, "unknown dynamics model");
    }
    if (!finite_all(d->A_dyn, n_models * ns * ns) || !finite_all(d->B_dyn, n_models * ns * nu) ||
        !finite_all(d->c_dyn, n_models * ns) || !finite_all(d->Q_s, (long long)ns * ns) || !finite_all(d->Q_u, (long long)nu * nu) ||
        !finite_all(d->x_ref, (long long)d->n_scen * (N + 1) * ns) || !finite_all(d->x0, (long long)d->n_scen * ns))
        return fail(CADMM_INVALID, "non-finite model, cost or reference");
    if (!(d->sigma > 0) || !(d->eps_prox > 0) || !std::isfinite(d->sigma) || !std::isfinite(d->eps_prox) ||
        !std::isfinite(d->eps_pri) || !std::isfinite(d->eps_dual))
        return fail(CADMM_INVALID, "sigma and eps_prox must be finite and > 0, eps_pri/eps_dual finite");
    if (M > 0 && !pair_variant_supported(dim, max_pf, max_of))
        return fail(CADMM_INVALID, "face counts exceed the compiled kernel variants");
    if (d->waves_per_group < 0 || d->waves_per_group > kMaxWavesPerGroup)
        return fail(CADMM_INVALID, "waves_per_group out of range (0..8)");
    if (d->lanes_per_pair != 0 && d->lanes_per_pair != 1 && d->lanes_per_pair != 2 && d->lanes_per_pair != 4)
        return fail(CADMM_INVALID, "lanes_per_pair must be 0 (autotune), 1, 2 or 4");
    if (d->max_sweeps < 0 || d->max_sweeps > 1000) return fail(CADMM_INVALID, "max_sweeps out of range");
    // state and input bounds: NaN-free, min <= max, any finite entry turns them on
    int has_bounds = 0;
    for (int kind = 0; kind < 2; ++kind) {
        const double* lo = kind == 0 ? d->s_min : d->u_min;
        const double* hi = kind == 0 ? d->s_max : d->u_max;
        const int n = kind == 0 ? ns : nu;
        for (int i = 0; i < n; ++i) {
            const double l = lo ? lo[i] : -INFINITY, u = hi ? hi[i] : INFINITY;
            if (std::isnan(l) || std::isnan(u) || l > u || l == INFINITY || u == -INFINITY)
                return fail(CADMM_INVALID, "state/input bounds: NaN, +inf lower, -inf upper or min > max");
            if (std::isfinite(l) || std::isfinite(u)) has_bounds = 1;
        }
    }
    if (has_bounds && !bounds_supported(ns, nu))
        return fail(CADMM_INVALID, "state/input bounds need n_s <= 12 and n_u <= 4");

    L.dim = dim; L.n_s = ns; L.n_u = nu; L.N = N; L.n_parts = d->n_parts; L.n_scen = d->n_scen;
    L.M = M; L.Fr = Fr; L.Fo = Fo; L.n_att = n_att; L.nq = dim + n_att; L.nc = L.nq * (L.nq + 1) / 2 + L.nq;
    L.max_pf = max_pf; L.max_of = max_of;
    L.n_blocks = d->n_parts * M;
    L.n_pairs = (long long)L.n_blocks * N;
    long long yf = 0;
    for (int s = 0; s < d->n_scen; ++s)
        for (int i = 0; i < d->n_parts; ++i)
            for (int j = d->obs_ptr[s]; j < d->obs_ptr[s + 1]; ++j)
                yf += (long long)((d->part_face_ptr[i + 1] - d->part_face_ptr[i]) +
                                  (d->obs_face_ptr[j + 1] - d->obs_face_ptr[j]) + 1) * N;
    if (yf >= (1LL << 31)) return fail(CADMM_INVALID, "problem too large (dual variables exceed 2^31 floats)");
    L.y_floats = yf;

    size_t off = 0;
    const int nb = std::max(L.n_blocks, 1);
    L.part_faces = take(off, sizeof(float4) * Fr);
    L.part_face_ptr = take(off, sizeof(int) * (d->n_parts + 1));
    L.part_off = take(off, sizeof(float) * 3 * d->n_parts);
    L.obs_faces = take(off, sizeof(float4) * std::max(Fo, 1));
    L.obs_d64 = take(off, sizeof(double) * std::max(Fo, 1));
    L.obs_dc = take(off, sizeof(float4) * std::max(Fo, 1));
    L.obs_face_ptr = take(off, sizeof(int) * (M + 1));
    L.blocks = take(off, sizeof(int4) * nb);
    L.block_yoff = take(off, sizeof(int) * nb);
    L.bdesc = take(off, sizeof(int4) * nb);
    L.wg_items = take(off, sizeof(int4) * nb);
    L.scen_wg = take(off, sizeof(int2) * d->n_scen);
    L.n_models = n_models;
    L.A_dyn = take(off, sizeof(float) * n_models * ns * ns);
    L.B_dyn = take(off, sizeof(float) * n_models * ns * nu);
    L.c_dyn = take(off, sizeof(float) * n_models * ns);
    const size_t n_lin = d->model != CADMM_MODEL_LINEAR ? (size_t)d->n_scen * N : 1;
    L.A_lin = take(off, sizeof(float) * n_lin * ns * ns);
    L.B_lin = take(off, sizeof(float) * n_lin * ns * nu);
    L.Q_s = take(off, sizeof(float) * ns * ns);
    L.Q_u = take(off, sizeof(float) * nu * nu);
    L.x_ref = take(off, sizeof(float) * d->n_scen * (N + 1) * ns);
    L.x0 = take(off, sizeof(float) * d->n_scen * ns);
    L.x = take(off, sizeof(float) * d->n_scen * (N + 1) * ns);
    L.u = take(off, sizeof(float) * d->n_scen * N * nu);
    L.y = take(off, sizeof(float) * std::max<long long>(yf, 1));
    L.zeta = take(off, sizeof(float) * std::max<long long>(L.n_pairs, 1));
    L.xi = take(off, sizeof(float) * std::max<long long>(L.n_pairs * dim, 1));
    L.y_snap = take(off, sizeof(float) * std::max<long long>(yf, 1));
    L.x_snap = take(off, sizeof(float) * d->n_scen * (N + 1) * ns);
    L.u_snap = take(off, sizeof(float) * d->n_scen * N * nu);
    L.contrib = take(off, sizeof(float) * (size_t)nb * L.nc * 64);
    L.rdual_part = take(off, sizeof(float) * nb);
    L.rpri_part = take(off, sizeof(float) * nb);
    L.unconv_part = take(off, sizeof(int) * nb);
    L.r_pri = take(off, sizeof(float) * d->n_scen);
    L.r_dual = take(off, sizeof(float) * d->n_scen);
    L.done = take(off, sizeof(int) * d->n_scen);
    L.iters = take(off, sizeof(int) * d->n_scen);
    L.unconv = take(off, sizeof(int) * d->n_scen);
    L.hist_pri = take(off, sizeof(float) * (size_t)kHistCap * d->n_scen);
    L.hist_dual = take(off, sizeof(float) * (size_t)kHistCap * d->n_scen);
    L.has_bounds = has_bounds;
    L.blim = take(off, sizeof(float) * 2 * (ns + nu));
    L.hq_b = take(off, has_bounds ? sizeof(float) * (size_t)d->n_scen * N * L.nc : 0);
    L.bW = take(off, has_bounds ? sizeof(float) * 2 * (size_t)d->n_scen * kBoundSlots * N * (ns + nu) : 0);
    L.bstat = take(off, sizeof(int) * d->n_scen);
    L.bprev = take(off, sizeof(int) * (size_t)d->n_scen * (kBoundSlots + 1));
    L.hq_pre = take(off, sizeof(float) * (size_t)d->n_scen * N * L.nc);
    L.alpha = take(off, sizeof(float) * std::max<long long>(L.n_pairs, 1));
    L.cost = take(off, sizeof(float) * d->n_scen);
    L.min_alpha = take(off, sizeof(float) * d->n_scen);
    L.total = (off + 255) & ~size_t(255);
    return CADMM_OK;
}

}  // namespace

struct cadmm_handle {
    Layout L;
    DevProblem P;
    char* ws;
    hipStream_t stream;
    hipGraphExec_t g1, gK;       // 1-iteration and kGraphBlock-iteration graphs
    hipGraphExec_t g1n, gKn;     // the same without the stopping test (unrolled runs)
    int W, G, grid;             // pair blocks and lanes per pair of the pair-phase launch
    // the last recorded unrolled run (admm_record), consumed by admm_backward
    int rec_iters, rec_every;
    void* rec_ws;
    size_t rec_bytes;
    std::vector<int> obs_ptr;    // host copy (scenario -> obstacles)
    int* hdone;                  // pinned host copies of the done flags, [2][n_scen] (admm_solve)
    hipEvent_t ev_done[2];       // recorded behind each copy
    std::vector<int4> blocks;    // host copy
};

namespace {

template <class T>
T* at(cadmm_handle* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

// work lists for W waves (= pair blocks) per workgroup; workgroups never
// straddle scenarios so per-step sums stay per scenario.
void build_worklists(const Layout& L, const std::vector<int>& obs_ptr, int W, std::vector<int4>& items,
                     std::vector<int2>& scen_wg)
{
    items.clear();
    scen_wg.assign(L.n_scen, int2{0, 0});
    int b = 0;
    for (int s = 0; s < L.n_scen; ++s) {
        const int nb_s = L.n_parts * (obs_ptr[s + 1] - obs_ptr[s]);
        scen_wg[s].x = (int)items.size();
        int k = 0;
        for (int b0 = 0; b0 < nb_s; b0 += W, ++k) items.push_back(int4{s, b + b0, b + std::min(nb_s, b0 + W), k});
        scen_wg[s].y = (int)items.size();
        b += nb_s;
    }
}

int upload_worklists(cadmm_handle* h, int W)
{
    std::vector<int4> items;
    std::vector<int2> sw;
    build_worklists(h->L, h->obs_ptr, W, items, sw);
    if (!items.empty())
        HIP_TRY(hipMemcpyAsync(h->ws + h->L.wg_items, items.data(), sizeof(int4) * items.size(),
                               hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->ws + h->L.scen_wg, sw.data(), sizeof(int2) * sw.size(), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->W = W;
    h->P.n_wg = (int)items.size();
    // scenarios with many pair-phase workgroups: their per-step sums are
    // spread over many workgroups by a kernel of their own (one trajectory
    // workgroup reading every partial would be bound by one CU's bandwidth)
    h->P.hq_pre = h->P.n_wg >= kPreSumWorkgroups * h->L.n_scen ? at<float>(h, h->L.hq_pre) : nullptr;
    h->grid = std::max(1, h->P.n_wg);
    return CADMM_OK;
}

// one ADMM iteration: (1) pair QPs + contributions, (2) trajectory QP,
// (3) multiplier update, residual sums and stopping test
int enqueue_iteration(cadmm_handle* h, hipStream_t st, bool stop_test = true, float* hq_save = nullptr)
{
    if (h->L.n_blocks > 0) HIP_TRY(launch_pair_phase(h->P, h->W, h->G, h->grid, st));
    // without pair blocks the LQ of a linear model is its own fixed point
    // (solved from base 0); a nonlinear model is relinearised every iteration
    const int no_pairs = h->L.n_blocks == 0 && h->P.model == CADMM_MODEL_LINEAR;
    HIP_TRY(launch_traj_phase(h->P, no_pairs, st, hq_save));
    if (h->L.n_blocks > 0) HIP_TRY(launch_mult_phase(h->P, h->W, h->grid, st));
    if (stop_test) HIP_TRY(launch_residual(h->P, st));
    return CADMM_OK;
}

int capture(cadmm_handle* h, hipStream_t cap, int iters, hipGraphExec_t* out, bool stop_test = true)
{
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    int rc = CADMM_OK;
    for (int i = 0; i < iters && rc == CADMM_OK; ++i) rc = enqueue_iteration(h, cap, stop_test);
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (rc != CADMM_OK) return rc;
    if (e != hipSuccess) return fail(CADMM_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CADMM_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return CADMM_OK;
}

void drop_graphs(cadmm_handle* h)
{
    for (hipGraphExec_t* g : {&h->g1, &h->gK, &h->g1n, &h->gKn}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
}

// everything the handle owns besides the caller's workspace and stream
void release(cadmm_handle* h)
{
    drop_graphs(h);
    for (hipEvent_t& e : h->ev_done)
        if (e) (void)hipEventDestroy(e);
    if (h->hdone) (void)hipHostFree(h->hdone);
    delete h;
}

// The four graphs are captured on a stream of their own (capture cannot
// run on a caller's legacy default stream), created for the capture and
// destroyed right after it: a handle keeps no stream besides the caller's.
int recapture(cadmm_handle* h)
{
    drop_graphs(h);
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    int rc;
    if ((rc = capture(h, cap, 1, &h->g1)) || (rc = capture(h, cap, kGraphBlock, &h->gK)) ||
        (rc = capture(h, cap, 1, &h->g1n, false)) || (rc = capture(h, cap, kGraphBlock, &h->gKn, false))) {
        (void)hipStreamDestroy(cap);
        return rc;
    }
    HIP_TRY(hipStreamDestroy(cap));
    return CADMM_OK;
}

// n iterations by graph replay, with or without the stopping test
int launch_graphs(cadmm_handle* h, int n, bool stop_test)
{
    hipGraphExec_t gk = stop_test ? h->gK : h->gKn, g1 = stop_test ? h->g1 : h->g1n;
    while (n >= kGraphBlock) {
        HIP_TRY(hipGraphLaunch(gk, h->stream));
        n -= kGraphBlock;
    }
    for (int i = 0; i < n; ++i) HIP_TRY(hipGraphLaunch(g1, h->stream));
    return CADMM_OK;
}

// ---- reverse pass: layout of the caller's gradient workspace ----
// An iterate slot holds (x, u, y, zeta, xi); u is kept because the
// trajectory QP is solved about (x^k, u^k), so a replay from a slot repeats
// the recorded run bit for bit. Checkpoint c holds the iterate k = c * every;
// the segment buffer holds the replayed iterates k0+1..k0+every of one
// segment (its iterate k0 is the checkpoint) and the stage sums of each
// replayed trajectory QP; 'fin' holds the last iterate.
struct Slot {
    size_t x, u, y, zeta, xi;
};

struct GradLayout {
    int iters, every, n_ckpt;
    std::vector<Slot> ckpt, seg;    // seg[0] unused (the checkpoint)
    std::vector<size_t> hq;
    Slot fin;
    size_t yb, zb, xib, qpart, w, gdb, gx0;
    size_t total;
};

GradLayout plan_grad(const Layout& L, int n_wg, int iters, int every)
{
    GradLayout G;
    G.iters = iters;
    G.every = std::min(every, iters);
    G.n_ckpt = (iters + G.every - 1) / G.every;
    size_t off = 0;
    const size_t xf = (size_t)L.n_scen * (L.N + 1) * L.n_s, uf = (size_t)L.n_scen * L.N * L.n_u;
    const size_t yf = std::max<long long>(L.y_floats, 1), pf = std::max<long long>(L.n_pairs, 1);
    auto slot = [&]() {
        Slot q;
        q.x = take(off, sizeof(float) * xf);
        q.u = take(off, sizeof(float) * uf);
        q.y = take(off, sizeof(float) * yf);
        q.zeta = take(off, sizeof(float) * pf);
        q.xi = take(off, sizeof(float) * pf * L.dim);
        return q;
    };
    for (int c = 0; c < G.n_ckpt; ++c) G.ckpt.push_back(slot());
    G.seg.push_back(Slot{0, 0, 0, 0, 0});
    for (int j = 1; j <= G.every; ++j) G.seg.push_back(slot());
    for (int j = 0; j < G.every; ++j) G.hq.push_back(take(off, sizeof(float) * (size_t)L.n_scen * L.N * L.nc));
    G.fin = slot();
    G.yb = take(off, sizeof(float) * yf);
    G.zb = take(off, sizeof(float) * pf);
    G.xib = take(off, sizeof(float) * pf * L.dim);
    G.qpart = take(off, sizeof(float) * (size_t)std::max(n_wg, 1) * L.nq * 64);
    G.w = take(off, sizeof(float) * (size_t)L.n_scen * L.N * L.n_s);
    G.gdb = take(off, sizeof(double) * (size_t)L.n_parts * std::max(L.Fo, 1));
    G.gx0 = take(off, sizeof(double) * (size_t)L.n_scen * L.n_s);
    G.total = (off + 255) & ~size_t(255);
    return G;
}

// copy the handle's iterate (x, u, y, zeta, xi) to or from a slot of base
int copy_slot(cadmm_handle* h, char* base, const Slot& q, bool to_slot)
{
    const Layout& L = h->L;
    const size_t xb = sizeof(float) * L.n_scen * (L.N + 1) * L.n_s, ub = sizeof(float) * L.n_scen * L.N * L.n_u,
                 yb = sizeof(float) * L.y_floats, zb = sizeof(float) * L.n_pairs,
                 ib = sizeof(float) * L.n_pairs * L.dim;
    const size_t hs[5] = {L.x, L.u, L.y, L.zeta, L.xi}, qs[5] = {q.x, q.u, q.y, q.zeta, q.xi},
                 nb[5] = {xb, ub, yb, zb, ib};
    for (int i = 0; i < 5; ++i) {
        if (nb[i] == 0) continue;
        void* dst = to_slot ? (void*)(base + qs[i]) : (void*)(h->ws + hs[i]);
        const void* src = to_slot ? (const void*)(h->ws + hs[i]) : (const void*)(base + qs[i]);
        HIP_TRY(hipMemcpyAsync(dst, src, nb[i], hipMemcpyDeviceToDevice, h->stream));
    }
    return CADMM_OK;
}

int fill_zero(void* p, size_t bytes, hipStream_t st)
{
    HIP_TRY(launch_fill(static_cast<float*>(p), (long long)(bytes / sizeof(float)), 0.f, st));
    return CADMM_OK;
}

// initial iterate (see collision_admm_setup)
int init_iterate(cadmm_handle* h)
{
    const Layout& L = h->L;
    hipStream_t st = h->stream;
    HIP_TRY(launch_fill(at<float>(h, L.zeta), L.n_pairs, 0.f, st));
    HIP_TRY(launch_fill(at<float>(h, L.xi), L.n_pairs * L.dim, 0.f, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.done), L.n_scen, 0, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.iters), L.n_scen, 0, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.unconv), L.n_scen, 0, st));
    HIP_TRY(launch_fill(at<float>(h, L.r_pri), L.n_scen, NAN, st));
    HIP_TRY(launch_fill(at<float>(h, L.r_dual), L.n_scen, NAN, st));
    HIP_TRY(launch_fill(at<float>(h, L.hist_pri), (long long)kHistCap * L.n_scen, NAN, st));
    HIP_TRY(launch_fill(at<float>(h, L.hist_dual), (long long)kHistCap * L.n_scen, NAN, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.bstat), L.n_scen, 0, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.bprev), (long long)L.n_scen * (kBoundSlots + 1), 0, st));
    HIP_TRY(launch_traj_phase(h->P, 1, st));
    if (L.n_blocks > 0) HIP_TRY(launch_init_pairs(h->P, nullptr, 1, st));
    return CADMM_OK;
}

// choose waves per workgroup by timing the pair phase and the trajectory
// phase (whose per-step reduction reads one partial per workgroup) from the
// same iterate
int autotune(cadmm_handle* h, int fixed_W, int fixed_G)
{
    const Layout& L = h->L;
    if (L.n_blocks == 0) {
        h->G = 1;
        return upload_worklists(h, 1);
    }
    hipStream_t st = h->stream;
    const size_t yb = sizeof(float) * L.y_floats, xb = sizeof(float) * L.n_scen * (L.N + 1) * L.n_s,
                 ub = sizeof(float) * L.n_scen * L.N * L.n_u;
    // time the candidates on an iterate of the running solve, not on the
    // initial one: the pair QPs of the first iterations are far easier (the
    // scale-LP certificates are near their optimum), so the initial iterate
    // misjudges the Newton sweeps the shapes have to carry
    int rc;
    if ((rc = upload_worklists(h, fixed_W > 0 ? fixed_W : 4))) return rc;
    h->G = fixed_G > 0 ? fixed_G : 1;
    if (!pair_group_supported(L.N, h->W, h->G)) {
        if ((rc = upload_worklists(h, 1))) return rc;
    }
    for (int i = 0; i < kTuneWarmIters; ++i)
        if ((rc = enqueue_iteration(h, st, false))) return rc;
    HIP_TRY(hipMemcpyAsync(h->ws + L.y_snap, h->ws + L.y, yb, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->ws + L.x_snap, h->ws + L.x, xb, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->ws + L.u_snap, h->ws + L.u, ub, hipMemcpyDeviceToDevice, st));
    auto restore = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(h->ws + L.y, h->ws + L.y_snap, yb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(h->ws + L.x, h->ws + L.x_snap, xb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(h->ws + L.u, h->ws + L.u_snap, ub, hipMemcpyDeviceToDevice, st));
        return CADMM_OK;
    };
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int Ws[] = {1, 2, 4, 8}, Gs[] = {1, 2, 4};
    float best = 1e30f;
    int bestW = 0, bestG = 1;
    for (int G : Gs) {
        if (fixed_G > 0 && G != fixed_G) continue;
        for (int W : Ws) {
            if (fixed_W > 0 && W != fixed_W) continue;
            if (!pair_group_supported(L.N, W, G)) continue;
            if (W > 1 && W / 2 >= L.n_blocks) continue;
            if ((rc = upload_worklists(h, W))) return rc;
            h->G = G;
            // sixteen iterations' pair and trajectory phases from the snapshot
            // (the spread of pair difficulty of a solve: shorter windows
            // ranked the lane-group sizes differently from whole solves),
            // best of two runs after one that warms caches and code
            float tot = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                if ((rc = restore())) return rc;
                HIP_TRY(hipEventRecord(e0, st));
                for (int k = 0; k < 16; ++k) {
                    HIP_TRY(launch_pair_phase(h->P, h->W, h->G, h->grid, st));
                    HIP_TRY(launch_traj_phase(h->P, 0, st));
                }
                HIP_TRY(hipEventRecord(e1, st));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) tot = std::min(tot, ms);
            }
            // a later shape has to win by 3%, so that run-to-run timing noise
            // does not flip the choice between near-equal shapes
            if (tot < 0.97f * best) { best = tot; bestW = W; bestG = G; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (bestW == 0) return fail(CADMM_INVALID, "no supported pair-kernel launch shape for this horizon");
    h->G = bestG;
    if ((rc = upload_worklists(h, bestW))) return rc;
    return init_iterate(h);   // back to the initial iterate of setup
}

}  // namespace

extern "C" {

const char* cadmm_strerror(int code)
{
    switch (code) {
    case CADMM_OK: return "ok";
    case CADMM_INVALID: return "invalid descriptor or argument";
    case CADMM_DEVICE: return "HIP device error";
    case CADMM_WORKSPACE: return "workspace too small or misaligned";
    case CADMM_NOT_CONVERGED: return "stopping test not met within the iteration budget (outputs written)";
    default: return "unknown status";
    }
}

const char* cadmm_last_error(void) { return g_last_error.c_str(); }

int cadmm_workspace_size(const cadmm_desc* desc, size_t* bytes, int* n_blocks, long long* n_pairs,
                         long long* y_floats)
{
    Layout L;
    int rc = validate_and_plan(desc, L);
    if (rc) return rc;
    if (bytes) *bytes = L.total;
    if (n_blocks) *n_blocks = L.n_blocks;
    if (n_pairs) *n_pairs = L.n_pairs;
    if (y_floats) *y_floats = L.y_floats;
    return CADMM_OK;
}

int collision_admm_setup(const cadmm_desc* d, void* d_ws, size_t bytes, hipStream_t stream, cadmm_handle** out)
{
    if (!out) return fail(CADMM_INVALID, "out handle pointer is NULL");
    *out = nullptr;
    Layout L;
    int rc = validate_and_plan(d, L);
    if (rc) return rc;
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
        return fail(CADMM_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
    if (bytes < L.total)
        return fail(CADMM_WORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");
    cadmm_handle* h = new cadmm_handle();
    h->L = L;
    h->ws = static_cast<char*>(d_ws);
    h->stream = stream;
    h->g1 = h->gK = h->g1n = h->gKn = nullptr;
    h->rec_iters = h->rec_every = 0;
    h->rec_ws = nullptr;
    h->rec_bytes = 0;
    h->obs_ptr.assign(d->obs_ptr, d->obs_ptr + d->n_scen + 1);
    h->hdone = nullptr;
    h->ev_done[0] = h->ev_done[1] = nullptr;
    auto bail = [&](int code) {
        release(h);
        return code;
    };
    if (hipHostMalloc(reinterpret_cast<void**>(&h->hdone), sizeof(int) * 2 * (size_t)d->n_scen) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_done[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_done[1], hipEventDisableTiming) != hipSuccess)
        return bail(fail(CADMM_DEVICE, "pinned host buffer or events for the stopping flags"));

    // ---- host staging (FP64 -> FP32, faces packed as float4) ----
    const int dim = L.dim, ns = L.n_s, nu = L.n_u, N = L.N;
    std::vector<float4> pf(L.Fr), of(std::max(L.Fo, 1));
    for (int k = 0; k < L.Fr; ++k)
        pf[k] = float4{(float)d->part_A[k * dim], (float)d->part_A[k * dim + 1],
                       dim == 3 ? (float)d->part_A[k * dim + 2] : 0.f, (float)d->part_b[k]};
    for (int k = 0; k < L.Fo; ++k)
        of[k] = float4{(float)d->obs_C[k * dim], (float)d->obs_C[k * dim + 1],
                       dim == 3 ? (float)d->obs_C[k * dim + 2] : 0.f, (float)d->obs_d[k]};
    // the rounding of each FP32 normal, kept for the FP64 face offsets
    std::vector<float4> dc(std::max(L.Fo, 1), float4{0.f, 0.f, 0.f, 0.f});
    for (int k = 0; k < L.Fo; ++k) {
        float e[3] = {0.f, 0.f, 0.f};
        for (int r = 0; r < dim; ++r) e[r] = (float)(d->obs_C[k * dim + r] - (double)(float)d->obs_C[k * dim + r]);
        dc[k] = float4{e[0], e[1], e[2], 0.f};
    }
    std::vector<float> poff(3 * L.n_parts, 0.f);
    for (int i = 0; i < L.n_parts; ++i)
        for (int r = 0; r < dim; ++r) poff[i * 3 + r] = (float)d->part_off[i * dim + r];
    std::vector<int4> blocks, bdesc;
    std::vector<int> yoff;
    long long off = 0;
    for (int s = 0; s < L.n_scen; ++s)
        for (int i = 0; i < L.n_parts; ++i)
            for (int j = d->obs_ptr[s]; j < d->obs_ptr[s + 1]; ++j) {
                const int nr = d->part_face_ptr[i + 1] - d->part_face_ptr[i];
                const int no = d->obs_face_ptr[j + 1] - d->obs_face_ptr[j];
                const int n = nr + no + 1;
                blocks.push_back(int4{s, i, j, n});
                // face counts fit 8 bits (the compiled pair kernels take at most 32) and
                // part indices 16 (checked with the descriptor)
                bdesc.push_back(int4{d->part_face_ptr[i], d->obs_face_ptr[j], (int)off, nr | (no << 8) | (i << 16)});
                yoff.push_back((int)off);
                off += (long long)n * N;
            }
    h->blocks = blocks;
    auto f32 = [](const double* p, size_t n) {
        std::vector<float> v(n);
        for (size_t i = 0; i < n; ++i) v[i] = (float)p[i];
        return v;
    };
    const size_t nm = (size_t)L.n_models;
    std::vector<float> Ad = f32(d->A_dyn, nm * ns * ns), Bd = f32(d->B_dyn, nm * ns * nu), cd = f32(d->c_dyn, nm * ns),
                       Qs = f32(d->Q_s, ns * ns), Qu = f32(d->Q_u, nu * nu),
                       xr = f32(d->x_ref, (size_t)L.n_scen * (N + 1) * ns), x0 = f32(d->x0, (size_t)L.n_scen * ns);
    // bounds as (s_min, s_max, u_min, u_max), +-inf where absent
    std::vector<float> blim(2 * (ns + nu));
    for (int i = 0; i < ns; ++i) {
        blim[i] = d->s_min ? (float)d->s_min[i] : -INFINITY;
        blim[ns + i] = d->s_max ? (float)d->s_max[i] : INFINITY;
    }
    for (int j = 0; j < nu; ++j) {
        blim[2 * ns + j] = d->u_min ? (float)d->u_min[j] : -INFINITY;
        blim[2 * ns + nu + j] = d->u_max ? (float)d->u_max[j] : INFINITY;
    }
    auto up = [&](size_t o, const void* src, size_t nbytes) -> int {
        if (nbytes == 0) return CADMM_OK;
        HIP_TRY(hipMemcpyAsync(h->ws + o, src, nbytes, hipMemcpyHostToDevice, stream));
        return CADMM_OK;
    };
    if ((rc = up(L.part_faces, pf.data(), sizeof(float4) * L.Fr)) ||
        (rc = up(L.part_face_ptr, d->part_face_ptr, sizeof(int) * (L.n_parts + 1))) ||
        (rc = up(L.part_off, poff.data(), sizeof(float) * poff.size())) ||
        (rc = up(L.obs_faces, of.data(), sizeof(float4) * L.Fo)) ||
        (rc = up(L.obs_d64, d->obs_d, sizeof(double) * L.Fo)) ||
        (rc = up(L.obs_dc, dc.data(), sizeof(float4) * dc.size())) ||
        (rc = up(L.obs_face_ptr, d->obs_face_ptr, sizeof(int) * (L.M + 1))) ||
        (rc = up(L.blocks, blocks.data(), sizeof(int4) * blocks.size())) ||
        (rc = up(L.block_yoff, yoff.data(), sizeof(int) * yoff.size())) ||
        (rc = up(L.bdesc, bdesc.data(), sizeof(int4) * bdesc.size())) ||
        (rc = up(L.A_dyn, Ad.data(), sizeof(float) * Ad.size())) ||
        (rc = up(L.B_dyn, Bd.data(), sizeof(float) * Bd.size())) ||
        (rc = up(L.c_dyn, cd.data(), sizeof(float) * cd.size())) ||
        (rc = up(L.Q_s, Qs.data(), sizeof(float) * Qs.size())) ||
        (rc = up(L.Q_u, Qu.data(), sizeof(float) * Qu.size())) ||
        (rc = up(L.x_ref, xr.data(), sizeof(float) * xr.size())) ||
        (rc = up(L.x0, x0.data(), sizeof(float) * x0.size())) ||
        (rc = up(L.blim, blim.data(), sizeof(float) * blim.size())))
        return bail(rc);
    // host staging buffers must stay alive until the copies complete
    if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(CADMM_DEVICE, "upload failed"));

    DevProblem& P = h->P;
    std::memset(&P, 0, sizeof(P));
    P.dim = dim; P.n_s = ns; P.n_u = nu; P.N = N; P.n_parts = L.n_parts; P.n_scen = L.n_scen;
    P.n_blocks = L.n_blocks; P.att_kind = d->att_kind; P.n_att = L.n_att; P.nq = L.nq; P.nc = L.nc;
    for (int r = 0; r < dim; ++r) P.pos_idx[r] = d->pos_idx[r];
    for (int a = 0; a < L.n_att; ++a) P.att_idx[a] = d->att_idx[a];
    P.sigma = (float)d->sigma; P.eps_prox = (float)d->eps_prox;
    P.eps_pri = (float)d->eps_pri; P.eps_dual = (float)d->eps_dual;
    P.max_sweeps = d->max_sweeps > 0 ? d->max_sweeps : 24;
    P.max_part_faces = L.max_pf; P.max_obs_faces = L.max_of;
    P.part_faces = at<float4>(h, L.part_faces);
    P.part_face_ptr = at<int>(h, L.part_face_ptr);
    P.part_off = at<float>(h, L.part_off);
    P.obs_faces = at<float4>(h, L.obs_faces);
    P.obs_d64 = at<double>(h, L.obs_d64);
    P.obs_dc = at<float4>(h, L.obs_dc);
    P.obs_face_ptr = at<int>(h, L.obs_face_ptr);
    P.blocks = at<int4>(h, L.blocks);
    P.block_yoff = at<int>(h, L.block_yoff);
    P.bdesc = at<int4>(h, L.bdesc);
    P.wg_items = at<int4>(h, L.wg_items);
    P.scen_wg = at<int2>(h, L.scen_wg);
    P.A_dyn = at<float>(h, L.A_dyn); P.B_dyn = at<float>(h, L.B_dyn); P.c_dyn = at<float>(h, L.c_dyn);
    P.dyn_ts = d->dyn_t_stride; P.dyn_ss = d->dyn_s_stride; P.model = d->model;
    for (int k = 0; k < 8; ++k) P.model_par[k] = d->model_par[k];
    P.A_lin = at<float>(h, L.A_lin); P.B_lin = at<float>(h, L.B_lin);
    P.Q_s = at<float>(h, L.Q_s); P.Q_u = at<float>(h, L.Q_u);
    P.x_ref = at<float>(h, L.x_ref); P.x0 = at<float>(h, L.x0);
    P.x = at<float>(h, L.x); P.u = at<float>(h, L.u); P.y = at<float>(h, L.y);
    P.zeta = at<float>(h, L.zeta); P.xi = at<float>(h, L.xi);
    P.contrib = at<float>(h, L.contrib);
    P.rdual_part = at<float>(h, L.rdual_part); P.rpri_part = at<float>(h, L.rpri_part);
    P.unconv_part = at<int>(h, L.unconv_part);
    P.r_pri = at<float>(h, L.r_pri); P.r_dual = at<float>(h, L.r_dual);
    P.done = at<int>(h, L.done); P.iters = at<int>(h, L.iters); P.unconv = at<int>(h, L.unconv);
    P.hist_pri = at<float>(h, L.hist_pri); P.hist_dual = at<float>(h, L.hist_dual); P.hist_cap = kHistCap;
    P.has_bounds = L.has_bounds;
    P.xlo = at<float>(h, L.blim); P.xhi = P.xlo + ns; P.ulo = P.xlo + 2 * ns; P.uhi = P.ulo + nu;
    P.hq_b = L.has_bounds ? at<float>(h, L.hq_b) : nullptr;
    P.bW = L.has_bounds ? at<float>(h, L.bW) : nullptr;
    P.bstat = at<int>(h, L.bstat);
    P.bprev = at<int>(h, L.bprev);

    h->G = d->lanes_per_pair > 0 ? d->lanes_per_pair : 1;
    if ((rc = upload_worklists(h, d->waves_per_group > 0 ? d->waves_per_group : 1))) return bail(rc);
    if ((rc = init_iterate(h))) return bail(rc);
    if (L.n_blocks > 0 && d->waves_per_group > 0 && d->lanes_per_pair > 0) {
        if (!pair_group_supported(L.N, d->waves_per_group, d->lanes_per_pair))
            return bail(fail(CADMM_INVALID, "waves_per_group x waves per block exceeds 8 for this horizon"));
    } else if ((rc = autotune(h, d->waves_per_group, d->lanes_per_pair))) {
        return bail(rc);
    }
    if ((rc = recapture(h))) return bail(rc);
    if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(CADMM_DEVICE, "setup failed"));
    *out = h;
    return CADMM_OK;
}

int admm_iterate(cadmm_handle* h, int n_iters)
{
    if (!h || n_iters < 0) return fail(CADMM_INVALID, "bad handle or iteration count");
    return launch_graphs(h, n_iters, true);
}

int admm_reset(cadmm_handle* h)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    return init_iterate(h);
}

int admm_solve(cadmm_handle* h, int max_iters, int check_every, cadmm_result* out)
{
    if (!h || max_iters < 0) return fail(CADMM_INVALID, "bad handle or iteration count");
    const Layout& L = h->L;
    if (check_every <= 0) check_every = kGraphBlock;
    std::vector<int> done(L.n_scen, 0);
    // chunks of check_every iterations, each followed by a copy of the done
    // flags into pinned memory and an event; chunk c + 1 is queued before the
    // flags of chunk c are read, so the GPU never waits for the host. Once
    // every scenario has stopped, the chunk already queued runs as no-ops
    // (the kernels skip stopped scenarios), so results do not depend on it.
    int it = 0;
    auto queue_chunk = [&](int c) -> int {
        const int chunk = std::min(check_every, max_iters - it);
        int rc = admm_iterate(h, chunk);
        if (rc) return rc;
        it += chunk;
        HIP_TRY(hipMemcpyAsync(h->hdone + (size_t)(c & 1) * L.n_scen, h->ws + L.done, sizeof(int) * L.n_scen,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipEventRecord(h->ev_done[c & 1], h->stream));
        return CADMM_OK;
    };
    if (max_iters > 0) {
        int rc = queue_chunk(0);
        if (rc) return rc;
        for (int c = 0;; ++c) {
            const bool more = it < max_iters;
            if (more && (rc = queue_chunk(c + 1))) return rc;
            HIP_TRY(hipEventSynchronize(h->ev_done[c & 1]));
            bool all = true;
            for (int s = 0; s < L.n_scen; ++s) all &= h->hdone[(size_t)(c & 1) * L.n_scen + s] != 0;
            if (all || !more) break;
        }
    }
    // final certificate and cost
    HIP_TRY(launch_cost(h->P, at<float>(h, L.cost), h->stream));
    if (L.n_blocks > 0) {
        HIP_TRY(launch_init_pairs(h->P, at<float>(h, L.alpha), 0, h->stream));
        HIP_TRY(launch_min_alpha(h->P, at<float>(h, L.alpha), at<float>(h, L.min_alpha), h->stream));
    } else {
        HIP_TRY(launch_fill(at<float>(h, L.min_alpha), L.n_scen, INFINITY, h->stream));
    }
    std::vector<float> rp(L.n_scen), rdv(L.n_scen), cost(L.n_scen), ma(L.n_scen);
    std::vector<int> iters(L.n_scen), unc(L.n_scen), bst(L.n_scen, 0);
    HIP_TRY(hipMemcpyAsync(rp.data(), h->ws + L.r_pri, sizeof(float) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(rdv.data(), h->ws + L.r_dual, sizeof(float) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(cost.data(), h->ws + L.cost, sizeof(float) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(ma.data(), h->ws + L.min_alpha, sizeof(float) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(iters.data(), h->ws + L.iters, sizeof(int) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(unc.data(), h->ws + L.unconv, sizeof(int) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(done.data(), h->ws + L.done, sizeof(int) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(bst.data(), h->ws + L.bstat, sizeof(int) * L.n_scen, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    bool all = true;
    for (int s = 0; s < L.n_scen; ++s) {
        if (out) {
            out[s].iters = iters[s];
            out[s].converged = done[s];
            out[s].r_pri = rp[s];
            out[s].r_dual = rdv[s];
            out[s].cost = cost[s];
            out[s].min_alpha = ma[s];
            out[s].unconverged_pairs = unc[s];
            out[s].active_bounds = bst[s];
        }
        all &= done[s] != 0;
    }
    return all ? CADMM_OK : CADMM_NOT_CONVERGED;
}

int admm_get_state(cadmm_handle* h, float* x, float* u, float* y, float* zeta, float* xi)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    const Layout& L = h->L;
    auto cp = [&](void* dst, size_t off, size_t nbytes) -> int {
        if (!dst || nbytes == 0) return CADMM_OK;
        HIP_TRY(hipMemcpyAsync(dst, h->ws + off, nbytes, hipMemcpyDeviceToDevice, h->stream));
        return CADMM_OK;
    };
    int rc;
    if ((rc = cp(x, L.x, sizeof(float) * L.n_scen * (L.N + 1) * L.n_s)) ||
        (rc = cp(u, L.u, sizeof(float) * L.n_scen * L.N * L.n_u)) ||
        (rc = cp(y, L.y, sizeof(float) * L.y_floats)) ||
        (rc = cp(zeta, L.zeta, sizeof(float) * L.n_pairs)) ||
        (rc = cp(xi, L.xi, sizeof(float) * L.n_pairs * L.dim)))
        return rc;
    return CADMM_OK;
}

int admm_set_state(cadmm_handle* h, const float* x, const float* u, const float* y, const float* zeta,
                   const float* xi)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    const Layout& L = h->L;
    auto cp = [&](const void* src, size_t off, size_t nbytes) -> int {
        if (!src || nbytes == 0) return CADMM_OK;
        HIP_TRY(hipMemcpyAsync(h->ws + off, src, nbytes, hipMemcpyDeviceToDevice, h->stream));
        return CADMM_OK;
    };
    int rc;
    if ((rc = cp(x, L.x, sizeof(float) * L.n_scen * (L.N + 1) * L.n_s)) ||
        (rc = cp(u, L.u, sizeof(float) * L.n_scen * L.N * L.n_u)) ||
        (rc = cp(y, L.y, sizeof(float) * L.y_floats)) ||
        (rc = cp(zeta, L.zeta, sizeof(float) * L.n_pairs)) ||
        (rc = cp(xi, L.xi, sizeof(float) * L.n_pairs * L.dim)))
        return rc;
    HIP_TRY(launch_fill_int(at<int>(h, L.done), L.n_scen, 0, h->stream));
    return CADMM_OK;
}

int admm_get_history(cadmm_handle* h, int max_rows, float* r_pri, float* r_dual)
{
    if (!h || max_rows < 0) return fail(CADMM_INVALID, "bad handle or size");
    const Layout& L = h->L;
    const int rows = std::min(max_rows, kHistCap);
    if (rows == 0) return 0;
    const size_t nbytes = sizeof(float) * (size_t)rows * L.n_scen;
    if (r_pri) HIP_TRY(hipMemcpyAsync(r_pri, h->ws + L.hist_pri, nbytes, hipMemcpyDeviceToHost, h->stream));
    if (r_dual) HIP_TRY(hipMemcpyAsync(r_dual, h->ws + L.hist_dual, nbytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return rows;
}

int admm_scales(cadmm_handle* h, float* alpha)
{
    if (!h || !alpha) return fail(CADMM_INVALID, "bad handle or output");
    if (h->L.n_blocks == 0) return CADMM_OK;
    HIP_TRY(launch_init_pairs(h->P, alpha, 0, h->stream));
    return CADMM_OK;
}

int admm_phase_times(cadmm_handle* h, int n_iters, float* ms_out)
{
    if (!h || n_iters <= 0 || !ms_out) return fail(CADMM_INVALID, "bad handle, count or output");
    // events recorded around each kernel's own execution (hipExtLaunchKernel),
    // a set per iteration, read after one synchronisation at the end, so that
    // the iterations run back to back
    std::vector<hipEvent_t> ev((size_t)8 * n_iters, nullptr);
    int rc = CADMM_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) { e = nullptr; rc = CADMM_DEVICE; }
    double acc[4] = {0, 0, 0, 0};
    hipStream_t st = h->stream;
    const bool pairs = h->L.n_blocks > 0;
    hipError_t err = hipSuccess;
    for (int it = 0; it < n_iters && rc == CADMM_OK && err == hipSuccess; ++it) {
        hipEvent_t* e = &ev[(size_t)8 * it];
        if (pairs) err = launch_pair_phase(h->P, h->W, h->G, h->grid, st, e[0], e[1]);
        if (err == hipSuccess)
            err = launch_traj_phase(h->P, !pairs && h->P.model == CADMM_MODEL_LINEAR, st, nullptr, e[2], e[3]);
        if (err == hipSuccess && pairs) err = launch_mult_phase(h->P, h->W, h->grid, st, e[4], e[5]);
        if (err == hipSuccess) err = launch_residual(h->P, st, e[6], e[7]);
    }
    if (rc == CADMM_OK && err == hipSuccess) err = hipStreamSynchronize(st);
    for (int it = 0; it < n_iters && rc == CADMM_OK && err == hipSuccess; ++it)
        for (int i = 0; i < 4 && err == hipSuccess; ++i) {
            if (!pairs && (i == 0 || i == 2)) continue;
            float ms = 0.f;
            err = hipEventElapsedTime(&ms, ev[(size_t)8 * it + 2 * i], ev[(size_t)8 * it + 2 * i + 1]);
            acc[i] += ms;
        }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != CADMM_OK) return fail(CADMM_DEVICE, "hipEventCreate failed");
    if (err != hipSuccess) return fail(CADMM_DEVICE, std::string("phase timing: ") + hipGetErrorString(err));
    for (int i = 0; i < 4; ++i) ms_out[i] = (float)(acc[i] / n_iters);
    return CADMM_OK;
}

int admm_launch_config(cadmm_handle* h, int* waves_per_group, int* n_workgroups, int* lanes_per_pair)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    if (waves_per_group) *waves_per_group = h->W;
    if (n_workgroups) *n_workgroups = h->P.n_wg;
    if (lanes_per_pair) *lanes_per_pair = h->G;
    return CADMM_OK;
}

int admm_set_params(cadmm_handle* h, const double* obs_d, const double* x0)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    const Layout& L = h->L;
    if (obs_d && !finite_all(obs_d, L.Fo)) return fail(CADMM_INVALID, "non-finite obstacle offsets");
    if (x0 && !finite_all(x0, (long long)L.n_scen * L.n_s)) return fail(CADMM_INVALID, "non-finite initial states");
    std::vector<float> x0f;
    if (obs_d && L.Fo > 0) {
        HIP_TRY(hipMemcpyAsync(h->ws + L.obs_d64, obs_d, sizeof(double) * L.Fo, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(launch_set_face_offsets(at<float4>(h, L.obs_faces), at<double>(h, L.obs_d64), L.Fo, h->stream));
    }
    if (x0) {
        x0f.resize((size_t)L.n_scen * L.n_s);
        for (size_t i = 0; i < x0f.size(); ++i) x0f[i] = (float)x0[i];
        HIP_TRY(hipMemcpyAsync(h->ws + L.x0, x0f.data(), sizeof(float) * x0f.size(), hipMemcpyHostToDevice,
                               h->stream));
    }
    // the host arrays must stay alive until the copies are done
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CADMM_OK;
}

int admm_reset_duals(cadmm_handle* h)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    const Layout& L = h->L;
    hipStream_t st = h->stream;
    HIP_TRY(launch_fill(at<float>(h, L.zeta), L.n_pairs, 0.f, st));
    HIP_TRY(launch_fill(at<float>(h, L.xi), L.n_pairs * L.dim, 0.f, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.done), L.n_scen, 0, st));
    if (L.n_blocks > 0) HIP_TRY(launch_init_pairs(h->P, nullptr, 1, st));
    return CADMM_OK;
}

int admm_set_reference(cadmm_handle* h, const double* x_ref)
{
    if (!h || !x_ref) return fail(CADMM_INVALID, "bad handle or NULL reference");
    const Layout& L = h->L;
    const size_t n = (size_t)L.n_scen * (L.N + 1) * L.n_s;
    if (!finite_all(x_ref, (long long)n)) return fail(CADMM_INVALID, "non-finite reference");
    std::vector<float> xr(n);
    for (size_t i = 0; i < n; ++i) xr[i] = (float)x_ref[i];
    HIP_TRY(hipMemcpyAsync(h->ws + L.x_ref, xr.data(), sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CADMM_OK;
}

int cadmm_model_step(int model, const double* model_par, const double* s, const double* u, double* s_next)
{
    if (model != CADMM_MODEL_BICYCLE && model != CADMM_MODEL_QUADROTOR)
        return fail(CADMM_INVALID, "cadmm_model_step needs a nonlinear model");
    if (!model_par || !s || !u || !s_next) return fail(CADMM_INVALID, "NULL argument");
    const int ns = model_ns(model), nu = model_nu(model);
    if (!finite_all(model_par, model == CADMM_MODEL_BICYCLE ? 2 : 6) || !finite_all(s, ns) || !finite_all(u, nu))
        return fail(CADMM_INVALID, "non-finite model parameters, state or input");
    double f[12];
    model_fc<double>(model, model_par, s, u, f);
    for (int i = 0; i < ns; ++i) s_next[i] = s[i] + model_par[0] * f[i];
    return CADMM_OK;
}

int admm_grad_workspace_size(cadmm_handle* h, int n_iters, int ckpt_every, size_t* bytes)
{
    if (!h || n_iters < 1 || ckpt_every < 1 || !bytes)
        return fail(CADMM_INVALID, "bad handle, iteration count, checkpoint interval or output");
    if (h->P.model != CADMM_MODEL_LINEAR || h->P.has_bounds)
        return fail(CADMM_INVALID, "the reverse pass needs the linear models and no state/input bounds");
    *bytes = plan_grad(h->L, h->P.n_wg, n_iters, ckpt_every).total;
    return CADMM_OK;
}

int admm_record(cadmm_handle* h, int n_iters, int ckpt_every, void* d_gws, size_t bytes, float* cost_out)
{
    if (!h || n_iters < 1 || ckpt_every < 1)
        return fail(CADMM_INVALID, "bad handle, iteration count or checkpoint interval");
    if (h->P.model != CADMM_MODEL_LINEAR || h->P.has_bounds)
        return fail(CADMM_INVALID, "the reverse pass needs the linear models and no state/input bounds");
    const Layout& L = h->L;
    const GradLayout G = plan_grad(L, h->P.n_wg, n_iters, ckpt_every);
    if (!d_gws || (reinterpret_cast<uintptr_t>(d_gws) & 255) != 0)
        return fail(CADMM_WORKSPACE, "gradient workspace must be a 256-byte aligned device pointer");
    if (bytes < G.total)
        return fail(CADMM_WORKSPACE, "gradient workspace too small: need " + std::to_string(G.total) + " bytes");
    char* base = static_cast<char*>(d_gws);
    hipStream_t st = h->stream;
    h->rec_iters = 0;
    // s^0 = obstacle-free LQ trajectory, zeta = xi = 0, y^0 as it stands
    HIP_TRY(launch_fill(at<float>(h, L.zeta), L.n_pairs, 0.f, st));
    HIP_TRY(launch_fill(at<float>(h, L.xi), L.n_pairs * L.dim, 0.f, st));
    HIP_TRY(launch_fill_int(at<int>(h, L.done), L.n_scen, 0, st));
    HIP_TRY(launch_traj_phase(h->P, 1, st));
    int rc;
    for (int c = 0; c < G.n_ckpt; ++c) {
        if ((rc = copy_slot(h, base, G.ckpt[c], true))) return rc;
        if ((rc = launch_graphs(h, std::min(G.every, n_iters - c * G.every), false))) return rc;
    }
    if ((rc = copy_slot(h, base, G.fin, true))) return rc;
    if (cost_out) HIP_TRY(launch_cost(h->P, cost_out, st));
    h->rec_iters = n_iters;
    h->rec_every = ckpt_every;
    h->rec_ws = d_gws;
    h->rec_bytes = bytes;
    return CADMM_OK;
}

int admm_backward(cadmm_handle* h, void* d_gws, size_t bytes, float dL_scale, float* grad_d, float* grad_x0)
{
    if (!h) return fail(CADMM_INVALID, "bad handle");
    if (h->P.model != CADMM_MODEL_LINEAR || h->P.has_bounds)
        return fail(CADMM_INVALID, "the reverse pass needs the linear models and no state/input bounds");
    if (h->rec_iters < 1 || d_gws != h->rec_ws || bytes < h->rec_bytes)
        return fail(CADMM_INVALID, "no recorded run in this gradient workspace (call admm_record first)");
    const Layout& L = h->L;
    if (!grad_x0 || (L.Fo > 0 && !grad_d)) return fail(CADMM_INVALID, "NULL gradient output");
    const GradLayout G = plan_grad(L, h->P.n_wg, h->rec_iters, h->rec_every);
    char* base = static_cast<char*>(d_gws);
    hipStream_t st = h->stream;
    const bool pairs = L.n_blocks > 0;
    int rc;
    if ((rc = fill_zero(base + G.yb, sizeof(float) * L.y_floats, st)) ||
        (rc = fill_zero(base + G.zb, sizeof(float) * L.n_pairs, st)) ||
        (rc = fill_zero(base + G.xib, sizeof(float) * L.n_pairs * L.dim, st)) ||
        (rc = fill_zero(base + G.gdb, sizeof(double) * L.n_parts * L.Fo, st)) ||
        (rc = fill_zero(base + G.gx0, sizeof(double) * L.n_scen * L.n_s, st)))
        return rc;
    HIP_TRY(launch_fill_int(at<int>(h, L.done), L.n_scen, 0, st));
    auto F = [&](size_t off) { return reinterpret_cast<float*>(base + off); };
    float* w = F(G.w);
    float* qpart = F(G.qpart);
    double* gx0 = reinterpret_cast<double*>(base + G.gx0);
    double* gdb = reinterpret_cast<double*>(base + G.gdb);
    bool first = true;
    for (int c = G.n_ckpt - 1; c >= 0; --c) {
        const int k0 = c * G.every, len = std::min(G.every, G.iters - k0);
        // replay the segment from its checkpoint, keeping every iterate and
        // the stage sums of every trajectory QP
        if ((rc = copy_slot(h, base, G.ckpt[c], false))) return rc;
        for (int j = 0; j < len; ++j) {
            if ((rc = enqueue_iteration(h, st, false, F(G.hq[j])))) return rc;
            if ((rc = copy_slot(h, base, G.seg[j + 1], true))) return rc;
        }
        for (int j = len - 1; j >= 0; --j) {
            const Slot& a = j == 0 ? G.ckpt[c] : G.seg[j];
            const Slot& n = G.seg[j + 1];
            // without pair blocks every trajectory QP is the obstacle-free one
            TrajAdjoint TA{pairs ? F(G.hq[j]) : nullptr, (first || !pairs) ? nullptr : qpart,
                           first ? F(G.fin.x) : nullptr,
                           first ? F(G.fin.u) : nullptr, w, gx0};
            HIP_TRY(launch_traj_adjoint(h->P, TA, st));
            PairAdjoint PA{F(a.x), F(n.x), F(a.y), F(n.y), F(a.zeta), F(a.xi), w, F(G.yb), F(G.zb), F(G.xib),
                           qpart, gdb, L.Fo, (k0 + j) >= 1 ? 1 : 0};
            HIP_TRY(launch_pair_adjoint(h->P, PA, h->W, h->grid, st));
            first = false;
        }
    }
    // s^0 = obstacle-free LQ(x_0)
    TrajAdjoint T0{nullptr, pairs ? qpart : nullptr, nullptr, nullptr, w, gx0};
    HIP_TRY(launch_traj_adjoint(h->P, T0, st));
    HIP_TRY(launch_grad_finalize(L.n_parts, L.Fo, gdb, L.n_scen * L.n_s, gx0, dL_scale, grad_d, grad_x0, st));
    // leave the handle at the last iterate of the recorded run
    if ((rc = copy_slot(h, base, G.fin, false))) return rc;
    return CADMM_OK;
}

void collision_admm_destroy(cadmm_handle* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    release(h);
}

namespace {
int check_pair_batch(const cadmm_pair_batch* b)
{
    if (!b) return fail(CADMM_INVALID, "batch is NULL");
    if (b->dim != 2 && b->dim != 3) return fail(CADMM_INVALID, "dim must be 2 or 3");
    if (b->n_pairs < 0) return fail(CADMM_INVALID, "n_pairs < 0");
    if (b->n_pairs == 0) return CADMM_OK;
    if (!b->row_ptr || !b->K || !b->kappa || !b->yhat || !b->bhat || !b->y || !b->r || !b->nu || !b->status)
        return fail(CADMM_INVALID, "NULL buffer");
    if (!(b->eps > 0.f)) return fail(CADMM_INVALID, "eps must be > 0");
    if (b->max_sweeps < 0) return fail(CADMM_INVALID, "max_sweeps < 0");
    return CADMM_OK;
}
}  // namespace

int pair_qp_batch_workspace_size(int n_pairs, size_t* bytes)
{
    if (n_pairs < 0 || !bytes) return fail(CADMM_INVALID, "n_pairs < 0 or NULL output");
    *bytes = pair_qp_batch_work_bytes(n_pairs);
    return CADMM_OK;
}

int pair_qp_batch_noalloc(const cadmm_pair_batch* b, hipStream_t stream)
{
    int rc = check_pair_batch(b);
    if (rc != CADMM_OK || b->n_pairs == 0) return rc;
    if (b->n_pairs > noalloc_max_pairs())
        return fail(CADMM_INVALID, "n_pairs exceeds the static buffer of pair_qp_batch_noalloc (" +
                                       std::to_string(noalloc_max_pairs()) + " pairs)");
    void* work = noalloc_scratch();
    if (!work) return fail(CADMM_DEVICE, "address of the static pair-batch buffer on this device");
    HIP_TRY(launch_pair_qp_batch(b->n_pairs, b->dim, b->row_ptr, b->K, b->kappa, b->yhat, b->bhat, b->eps,
                                 b->max_sweeps > 0 ? b->max_sweeps : 24, b->y, b->r, b->nu, b->status, stream,
                                 work));
    return CADMM_OK;
}

int pair_qp_batch(const cadmm_pair_batch* b, hipStream_t stream)
{
    int rc = check_pair_batch(b);
    if (rc != CADMM_OK || b->n_pairs == 0) return rc;
    if (b->solver == CADMM_PAIR_LEMKE) {
        HIP_TRY(launch_pair_qp_lemke(b->n_pairs, b->dim, b->row_ptr, b->K, b->kappa, b->yhat, b->bhat, b->eps,
                                     b->max_sweeps > 0 ? b->max_sweeps : 200, b->y, b->r, b->nu, b->status, stream));
        return CADMM_OK;
    }
    if (b->solver != CADMM_PAIR_NEWTON) return fail(CADMM_INVALID, "unknown pair solver");
    if (b->work) {
        if ((reinterpret_cast<uintptr_t>(b->work) & 255) != 0 || b->work_bytes < pair_qp_batch_work_bytes(b->n_pairs))
            return fail(CADMM_WORKSPACE, "pair-batch workspace misaligned or smaller than pair_qp_batch_workspace_size");
    }
    HIP_TRY(launch_pair_qp_batch(b->n_pairs, b->dim, b->row_ptr, b->K, b->kappa, b->yhat, b->bhat, b->eps,
                                 b->max_sweeps > 0 ? b->max_sweeps : 24, b->y, b->r, b->nu, b->status, stream,
                                 b->work));
    return CADMM_OK;
}

int pair_scale_batch(const cadmm_scale_batch* b, hipStream_t stream)
{
    if (!b) return fail(CADMM_INVALID, "batch is NULL");
    if (b->dim != 2 && b->dim != 3) return fail(CADMM_INVALID, "dim must be 2 or 3");
    if (b->n_pairs < 0) return fail(CADMM_INVALID, "n_pairs < 0");
    if (b->n_pairs == 0) return CADMM_OK;
    if (!b->a_ptr || !b->A || !b->b || !b->o_ptr || !b->Cp || !b->dp || !b->alpha || !b->lam || !b->mu || !b->status)
        return fail(CADMM_INVALID, "NULL buffer");
    HIP_TRY(launch_scale_batch(b->n_pairs, b->dim, b->a_ptr, b->A, b->b, b->o_ptr, b->Cp, b->dp, b->alpha, b->lam,
                               b->mu, b->status, stream));
    return CADMM_OK;
}

}  // extern "C"
