// gfx950 kernels of the stateless batch entry points of the collision-
// avoidance library (arXiv 2406.07048): many independent dual-update QPs
// (Sec. IV-C eq. const_least_square with the proximal term) and scale LPs
// (Sec. III-A eq. scale_opt, dual Sec. III-B eq. scale_opt_dual), with rows
// read from caller memory. One lane per problem.
#include "cadmm_solvers.h"

#include <algorithm>
#include <mutex>

namespace cadmm {

// ------------------------------------------------------------------------
// rows of the stateless batch, staged in LDS: per row (K_0..K_dim, kappa,
// yhat); the row scales 1 / (eps D) and ||K|| (D = ||K||^2) are formed in
// every solver pass (a few VALU instructions against an LDS tile of 5 floats
// a row instead of 7: 8 waves per CU instead of 5 to hide the LDS latency)
// ------------------------------------------------------------------------

// 1 / (eps D) and ||K|| = D rsq(D) of a row, D = ||K||^2, by the same
// instructions whether the row comes from LDS or from memory (a solve
// resumed in the second launch), so both see bitwise the same values.
// v_rcp_f32 / v_rsq_f32, about 1 ulp.
template <int C>
__device__ __forceinline__ void row_scales(const float (&k)[C], float eps, float& ie, float& kn)
{
    float D = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) D += k[c] * k[c];
    ie = __builtin_amdgcn_rcpf(eps * D);
    kn = D * __builtin_amdgcn_rsqf(fmaxf(D, 1e-30f));
}

// Row sources: the LDS tile of staged rows, or the caller's memory (a solve
// resumed in the second launch of the two-launch form) with the row scales
// formed as at staging.
template <int DIM>
struct LdsSrc {
    static constexpr int RW = DIM + 3;    // floats per staged row
    const float* rows;                    // LDS, RW floats per row
    float eps;

    __device__ __forceinline__ void load(int l, float (&k)[DIM + 1], float& kl, float& yh, float& ie,
                                         float& kn) const
    {
        const float* row = rows + l * RW;
#pragma unroll
        for (int c = 0; c <= DIM; ++c) k[c] = row[c];
        kl = row[DIM + 1];
        yh = row[DIM + 2];
        row_scales<DIM + 1>(k, eps, ie, kn);
    }
};

template <int DIM>
struct MemSrc {
    const float* K;
    const float* kap;
    const float* yhv;
    float eps;

    __device__ __forceinline__ void load(int l, float (&k)[DIM + 1], float& kl, float& yh, float& ie,
                                         float& kn) const
    {
#pragma unroll
        for (int c = 0; c <= DIM; ++c) k[c] = K[(size_t)l * (DIM + 1) + c];
        kl = kap[l];
        yh = yhv[l];
        row_scales<DIM + 1>(k, eps, ie, kn);
    }
};

template <int DIM, class Src>
struct BatchRows {
    static constexpr int NV = DIM + 2;
    int n;
    Src src;
    float bh[DIM + 1];

    // Gradient g and scale sc at z; with HESS the generalised Hessian of the
    // rows with y > 0 at z, with UNION of the rows with y > 0 at z or at zu.
    template <bool HESS, bool UNION = false>
    __device__ __forceinline__ void pass(const float (&z)[NV], float (&g)[NV], float (&H)[NV * NV],
                                         float& sc, const float* zu = nullptr) const
    {
        float gv[DIM + 1] = {}, gnu = 0.f, ysc = 0.f;
        if (HESS) {
#pragma unroll
            for (int i = 0; i < NV * NV; ++i) H[i] = 0.f;
        }
        for (int l = 0; l < n; ++l) {
            float k[DIM + 1], kl, yh, ie, kn;
            src.load(l, k, kl, yh, ie, kn);
            float s = -kl * z[DIM + 1];
#pragma unroll
            for (int c = 0; c <= DIM; ++c) s += k[c] * z[c];
            const float y = fmaxf(0.f, yh - s * ie);
#pragma unroll
            for (int c = 0; c <= DIM; ++c) gv[c] += y * k[c];
            gnu += kl * y;
            ysc += y * kn;
            bool on = y > 0.f;
            if (HESS && UNION) {
                float su = -kl * zu[DIM + 1];
#pragma unroll
                for (int c = 0; c <= DIM; ++c) su += k[c] * zu[c];
                on = on || yh - su * ie > 0.f;
            }
            if (HESS && on) {
                float w[NV];
#pragma unroll
                for (int c = 0; c <= DIM; ++c) w[c] = k[c];
                w[DIM + 1] = -kl;
#pragma unroll
                for (int r = 0; r < NV; ++r)
#pragma unroll
                    for (int c = r; c < NV; ++c) H[r * NV + c] += ie * w[r] * w[c];
            }
        }
        float mx = 0.f, bm = 0.f;
#pragma unroll
        for (int c = 0; c <= DIM; ++c) {
            g[c] = bh[c] - z[c] + gv[c];
            mx = fmaxf(mx, fabsf(z[c]));
            bm = fmaxf(bm, fabsf(bh[c]));
        }
        g[DIM + 1] = 1.f - gnu;
        sc = 1.f + bm + mx + ysc;
        if (HESS) {
#pragma unroll
            for (int c = 0; c <= DIM; ++c) H[c * NV + c] += 1.f;
            H[(DIM + 1) * NV + DIM + 1] += 1e-6f * (1.f + H[(DIM + 1) * NV + DIM + 1]);
#pragma unroll
            for (int r = 0; r < NV; ++r)
#pragma unroll
                for (int c = 0; c < r; ++c) H[r * NV + c] = H[c * NV + r];
        }
    }
};

// ------------------------------------------------------------------------
// stateless batch entry points
// ------------------------------------------------------------------------

// One wavefront per workgroup, one lane per pair: the workgroup's 64
// consecutive pairs own a contiguous row range, which is staged into the LDS
// tile with coalesced loads (in chunks of whole pairs when it exceeds the
// tile), solved from LDS, and the duals written back with coalesced stores.
// Every solver pass reads LDS instead of the caller's array-of-rows memory
// (read that way, the passes re-fetched their rows from HBM: 23x the bytes of
// one read per row, measured with FETCH_SIZE).
constexpr int kBatchPairs = 64;
constexpr int kBatchTileRows = 1024;   // > 64 pairs x the average rows; a pair holds at most 41

// The two-launch form: a wave runs as long as its slowest pair, so the first
// launch stops every solve after kStraggleSweeps sweeps and appends the
// unfinished ones (pair, Newton iterate and state) to a queue; a second
// launch, one lane per queued pair, resumes them where they stopped (the
// same iterates as an uninterrupted solve).
constexpr int kStraggleSweeps = 3;
constexpr int kEntryFloats = 12;       // pair, z (<= 5), gprev, al_prev, sweeps done; padded

template <int DIM>
__global__ void __launch_bounds__(kBatchPairs) pair_qp_batch_kernel(int n_pairs, const int* row_ptr, const float* K,
                                                                    const float* kappa, const float* yhat,
                                                                    const float* bhat, float eps, int max_sweeps,
                                                                    float* y, float* r, float* nu_out, int* status,
                                                                    int* qcount, float* queue)
{
    constexpr int NV = DIM + 2, C = DIM + 1;
    constexpr int RW = LdsSrc<DIM>::RW;
    static_assert(NV + 4 <= kEntryFloats, "queue entry too small");
    const int stop_at = queue ? kStraggleSweeps : 0x7fffffff;
    __shared__ float tile[kBatchTileRows * RW];
    const int lane = threadIdx.x;
    const int p0 = blockIdx.x * kBatchPairs;
    const int pend = min(p0 + kBatchPairs, n_pairs);
    const int p = p0 + lane;
    // row range of this lane's pair (lanes past the end hold an empty one)
    const int rb = row_ptr[min(p, pend)];
    const int re = __shfl_down(rb, 1, 64);
    const int rlast = row_ptr[pend];
    const int rend = lane == 63 ? rlast : re;
    const int n = p < pend ? rend - rb : 0;
    int pa = p0;
    while (pa < pend) {                    // uniform over the wave
        const int base = __shfl(rb, pa - p0, 64);
        // the chunk: whole pairs whose rows fit into the tile
        const bool fits = p >= pa && p < pend && rend - base <= kBatchTileRows;
        const unsigned long long m = __ballot(fits) >> (pa - p0);
        const int cnt = m == ~0ull >> (pa - p0) ? 64 - (pa - p0) : __builtin_ctzll(~m);
        if (cnt == 0) {
            // a pair with more rows than the tile (beyond the documented
            // limit of rows per pair): refused, the others go on
            if (p == pa) status[p] = -3;
            ++pa;
            continue;
        }
        const int pb = pa + cnt;
        const int nrows = __shfl(rend, pb - 1 - p0, 64) - base;
        for (int i = lane; i < nrows; i += kBatchPairs) {
            float* row = tile + i * RW;
            float kk[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                kk[c] = K[(size_t)(base + i) * C + c];
                row[c] = kk[c];
            }
            row[DIM + 1] = kappa[base + i];
            row[DIM + 2] = yhat[base + i];
        }
        __syncthreads();
        const bool act = p >= pa && p < pb;
        BatchRows<DIM, LdsSrc<DIM>> sr;
        float z[NV];
        NewtonState S;
        int sw = 0;
        if (act) {
            sr.n = n;
            sr.src.rows = tile + (rb - base) * RW;
            sr.src.eps = eps;
#pragma unroll
            for (int c = 0; c < C; ++c) sr.bh[c] = bhat[(size_t)p * C + c];
            // warm start v = K^T yhat + bhat; nu makes the largest kappa-row stationary
#pragma unroll
            for (int c = 0; c < C; ++c) z[c] = sr.bh[c];
            for (int l = 0; l < n; ++l) {
                const float* row = sr.src.rows + l * RW;
#pragma unroll
                for (int c = 0; c < C; ++c) z[c] += row[DIM + 2] * row[c];
            }
            float best = -1.f, nu = 0.f;
            for (int l = 0; l < n; ++l) {
                const float* row = sr.src.rows + l * RW;
                if (row[DIM + 1] > 0.f && row[DIM + 2] > best) {
                    best = row[DIM + 2];
                    float s = 0.f;
#pragma unroll
                    for (int c = 0; c < C; ++c) s += row[c] * z[c];
                    nu = s / row[DIM + 1];
                }
            }
            z[DIM + 1] = nu;
            sw = dual_newton<NV>(sr, z, max_sweeps, 1e-6f, S, stop_at);
        }
        // unfinished solves into the queue: one atomic per wave for its slots
        const bool paused = act && sw == kNewtonPaused;
        const unsigned long long pm = __ballot(paused);
        if (pm) {
            const int leader = __builtin_ctzll(pm);
            int qb = 0;
            if (lane == leader) qb = atomicAdd(qcount, __builtin_popcountll(pm));
            qb = __shfl(qb, leader, 64);
            if (paused) {
                const int slot = qb + __builtin_popcountll(pm & ((1ull << lane) - 1ull));
                float* ent = queue + (size_t)slot * kEntryFloats;
                ent[0] = __int_as_float(p);
#pragma unroll
                for (int i = 0; i < NV; ++i) ent[1 + i] = z[i];
                ent[NV + 1] = S.gprev;
                ent[NV + 2] = S.al_prev;
                ent[NV + 3] = __int_as_float(S.it);
            }
        }
        if (act && !paused) {
            // primal rows: y over the staged yhat, r = K^T y + bhat
            float rr[C];
#pragma unroll
            for (int c = 0; c < C; ++c) rr[c] = sr.bh[c];
            for (int l = 0; l < n; ++l) {
                float* row = tile + (rb - base + l) * RW;
                float kk[C], ie, kn;
#pragma unroll
                for (int c = 0; c < C; ++c) kk[c] = row[c];
                row_scales<C>(kk, eps, ie, kn);
                float s = -row[DIM + 1] * z[DIM + 1];
#pragma unroll
                for (int c = 0; c < C; ++c) s += row[c] * z[c];
                const float yl = fmaxf(0.f, row[DIM + 2] - s * ie);
                row[DIM + 2] = yl;
#pragma unroll
                for (int c = 0; c < C; ++c) rr[c] += yl * row[c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) r[(size_t)p * C + c] = rr[c];
            nu_out[p] = z[DIM + 1];
            status[p] = sw;
        }
        __syncthreads();
        for (int i = lane; i < nrows; i += kBatchPairs) y[base + i] = tile[i * RW + DIM + 2];
        __syncthreads();
        pa = pb;
    }
}

// Second launch of the two-launch form: one lane per queued pair resumes its
// solve from the saved iterate and state, reading its rows from memory with
// the row scales formed as at staging, and writes its outputs. The queue
// length is the counter the first launch left; the grid strides over it.
template <int DIM>
__global__ void __launch_bounds__(kBatchPairs) pair_qp_straggle_kernel(const int* row_ptr, const float* K,
                                                                       const float* kappa, const float* yhat,
                                                                       const float* bhat, float eps, int max_sweeps,
                                                                       float* y, float* r, float* nu_out,
                                                                       int* status, const int* qcount,
                                                                       const float* queue)
{
    constexpr int NV = DIM + 2, C = DIM + 1;
    const int count = *qcount;
    for (int e = blockIdx.x * kBatchPairs + threadIdx.x; e < count; e += gridDim.x * kBatchPairs) {
        const float* ent = queue + (size_t)e * kEntryFloats;
        const int p = __float_as_int(ent[0]);
        const int r0 = row_ptr[p], n = row_ptr[p + 1] - r0;
        BatchRows<DIM, MemSrc<DIM>> gr;
        gr.n = n;
        gr.src.K = K + (size_t)r0 * C;
        gr.src.kap = kappa + r0;
        gr.src.yhv = yhat + r0;
        gr.src.eps = eps;
#pragma unroll
        for (int c = 0; c < C; ++c) gr.bh[c] = bhat[(size_t)p * C + c];
        float z[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) z[i] = ent[1 + i];
        NewtonState S;
        S.gprev = ent[NV + 1];
        S.al_prev = ent[NV + 2];
        S.it = __float_as_int(ent[NV + 3]);
        const int sw = dual_newton<NV>(gr, z, max_sweeps, 1e-6f, S, 0x7fffffff);
        float rr[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rr[c] = gr.bh[c];
        for (int l = 0; l < n; ++l) {
            float k[C], kl, yh, ie, kn;
            gr.src.load(l, k, kl, yh, ie, kn);
            float s = -kl * z[DIM + 1];
#pragma unroll
            for (int c = 0; c < C; ++c) s += k[c] * z[c];
            const float yl = fmaxf(0.f, yh - s * ie);
            y[r0 + l] = yl;
#pragma unroll
            for (int c = 0; c < C; ++c) rr[c] += yl * k[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) r[(size_t)p * C + c] = rr[c];
        nu_out[p] = z[DIM + 1];
        status[p] = sw;
    }
}

template <int DIM>
struct MemCols {
    int nr, no;
    const float* A;
    const float* b;
    const float* Cp;
    const float* dp;
    float cmx;
    __device__ int n() const { return nr + no; }
    __device__ float cmax() const { return cmx; }
    __device__ float cost(int j) const { return j < nr ? 0.f : dp[j - nr]; }
    __device__ void col(int j, float (&E)[DIM + 1]) const {
        if (j < nr) {
            E[0] = b[j];
#pragma unroll
            for (int q = 0; q < DIM; ++q) E[1 + q] = A[j * DIM + q];
        } else {
            E[0] = 0.f;
#pragma unroll
            for (int q = 0; q < DIM; ++q) E[1 + q] = Cp[(j - nr) * DIM + q];
        }
    }
};

template <int DIM>
__global__ void __launch_bounds__(256) scale_batch_kernel(int n_pairs, const int* a_ptr, const float* A,
                                                          const float* b, const int* o_ptr, const float* Cp,
                                                          const float* dp, float* alpha, float* lam,
                                                          float* mu, int* status)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    const int a0 = a_ptr[p], o0 = o_ptr[p];
    MemCols<DIM> mc;
    mc.nr = a_ptr[p + 1] - a0;
    mc.no = o_ptr[p + 1] - o0;
    mc.A = A + (size_t)a0 * DIM;
    mc.b = b + a0;
    mc.Cp = Cp + (size_t)o0 * DIM;
    mc.dp = dp + o0;
    float cm = 0.f;
    for (int l = 0; l < mc.no; ++l) cm = fmaxf(cm, fabsf(mc.dp[l]));
    mc.cmx = cm;
    float al, xB[DIM + 1];
    int basis[DIM + 1];
    const int st = revised_simplex<DIM>(mc, al, xB, basis);
    alpha[p] = al;
    for (int j = 0; j < mc.nr + mc.no; ++j) {
        float v = 0.f;
#pragma unroll
        for (int i = 0; i <= DIM; ++i) v = basis[i] == j ? xB[i] : v;
        if (j < mc.nr) lam[a0 + j] = v;
        else mu[o0 + j - mc.nr] = v;
    }
    status[p] = st;
}

hipError_t launch_pair_qp_batch(int n_pairs, int dim, const int* row_ptr, const float* K, const float* kappa,
                                const float* yhat, const float* bhat, float eps, int max_sweeps, float* y,
                                float* r, float* nu, int* status, hipStream_t st, void* work)
{
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (n_pairs + kBatchPairs - 1) / kBatchPairs;
    int* qcount = nullptr;
    float* queue = nullptr;
    if (work) {
        qcount = static_cast<int*>(work);
        queue = reinterpret_cast<float*>(static_cast<char*>(work) + 256);
        // the counter is cleared by a kernel, not a memset node
        hipError_t e = launch_fill_int(qcount, 1, 0, st);
        if (e != hipSuccess) return e;
    }
    if (dim == 2)
        hipLaunchKernelGGL(pair_qp_batch_kernel<2>, dim3(grid), dim3(kBatchPairs), 0, st, n_pairs, row_ptr, K,
                           kappa, yhat, bhat, eps, max_sweeps, y, r, nu, status, qcount, queue);
    else
        hipLaunchKernelGGL(pair_qp_batch_kernel<3>, dim3(grid), dim3(kBatchPairs), 0, st, n_pairs, row_ptr, K,
                           kappa, yhat, bhat, eps, max_sweeps, y, r, nu, status, qcount, queue);
    if (!work) return hipGetLastError();
    const int g2 = std::min(grid, 2048);
    if (dim == 2)
        hipLaunchKernelGGL(pair_qp_straggle_kernel<2>, dim3(g2), dim3(kBatchPairs), 0, st, row_ptr, K, kappa, yhat,
                           bhat, eps, max_sweeps, y, r, nu, status, qcount, queue);
    else
        hipLaunchKernelGGL(pair_qp_straggle_kernel<3>, dim3(g2), dim3(kBatchPairs), 0, st, row_ptr, K, kappa, yhat,
                           bhat, eps, max_sweeps, y, r, nu, status, qcount, queue);
    return hipGetLastError();
}

size_t pair_qp_batch_work_bytes(int n_pairs)
{
    return 256 + (size_t)std::max(n_pairs, 0) * kEntryFloats * sizeof(float);
}

// The library's own buffer of the two-launch form, for callers that cannot
// allocate: one copy per GPU (held until the process ends), found through
// its symbol address once per device, with that device current.
constexpr int kNoallocMaxPairs = 1 << 19;
static __device__ __align__(256) unsigned char scratch[256 + (size_t)kNoallocMaxPairs * kEntryFloats * sizeof(float)];

int noalloc_max_pairs() { return kNoallocMaxPairs; }

void* noalloc_scratch()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

hipError_t launch_scale_batch(int n_pairs, int dim, const int* a_ptr, const float* A, const float* b,
                              const int* o_ptr, const float* Cp, const float* dp, float* alpha, float* lam,
                              float* mu, int* status, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (n_pairs + 255) / 256;
    if (dim == 2)
        hipLaunchKernelGGL(scale_batch_kernel<2>, dim3(grid), dim3(256), 0, st, n_pairs, a_ptr, A, b, o_ptr, Cp,
                           dp, alpha, lam, mu, status);
    else
        hipLaunchKernelGGL(scale_batch_kernel<3>, dim3(grid), dim3(256), 0, st, n_pairs, a_ptr, A, b, o_ptr, Cp,
                           dp, alpha, lam, mu, status);
    return hipGetLastError();
}

}  // namespace cadmm
