// Batched GP / UPN: many independent reconstructions of uneven size solved
// together.  One round = gradient (where due), projected trial, transpose,
// projection, finalised sums, FP64 control, extrapolation -- each a single
// grouped launch over all problems -- captured once in a HIP graph and
// replayed.  The control kernel takes, per problem, exactly the decisions of
// the single-problem driver (BT test of Alg. 2 in Bregman form, mu estimate
// of eq. 9, theta root and beta of Alg. 3, gradient-map stop of Sec. III-D)
// with the same double arithmetic, so every problem follows the same
// iterates as its own tvreg_solve.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "host.hpp"
#include "raywalk.hpp"

namespace tvr {

namespace {

template <typename T>
__device__ void control_step(BatchProblem<T> &P)
{
    // no fused multiply-adds: every product and sum is rounded on its own,
    // as in the host driver, so both take identical decisions
#pragma clang fp contract(off)
    const double *S = P.sum;
    P.func_evals++;
    P.ry2_pending = 0;  // consumed by this round's finaliser
    const double xd2 = S[S_XD2];
    const double lhs = 0.5 * S[S_RD2] + P.alpha * S[S_BRB];
    const double phi_xb = 0.5 * S[S_R2] + P.alpha * S[S_TVB];
    P.ex = 0;
    const bool nest = P.method == TVREG_NESTEROV;  // given L: no line-search test
    if (!nest && lhs > 0.5 * P.L * xd2) {  // BT rejects: larger L, same gradient
        P.trials++;
        P.need_grad = 0;
        if (P.trials >= P.max_trials) {
            P.state = B_STALL;  // X keeps the last accepted point
            P.gm = P.L * sqrt(xd2);
            if (P.first) {
                P.gm0 = P.gm;
                P.iters = 1;
                P.mu = P.mu_bar > 0.0 ? P.mu_bar : 0.25 * P.L;
            } else {
                P.iters++;
            }
        } else {
            P.L *= P.rho;
        }
        return;
    }
    P.trials = 0;
    const double gm = P.L * sqrt(xd2);
    P.gm = gm;
    P.phi = phi_xb;
    T *t;
    const bool first = P.first != 0;
    if (first) {
        P.gm0 = gm;
        P.iters = 1;
        P.mu = nest ? P.mu_bar : (P.mu_bar > 0.0 ? P.mu_bar : 0.25 * P.L);
        P.theta = sqrt(P.mu / P.L);
        P.first = 0;
    } else {
        P.iters++;
    }
    const bool stop = P.stop_mode == 1 ? gm / (double)P.N <= P.eps
                                       : (P.gm0 == 0.0 || gm <= P.eps * P.gm0);
    // the accepted trial becomes X
    t = P.X;
    P.X = P.XB;
    P.XB = t;
    t = P.RX;
    P.RX = P.RXB;
    P.RXB = t;
    if (stop) {
        P.state = B_CONVERGED;
        P.need_grad = 0;
        return;
    }
    if ((P.method == TVREG_UPN || nest) && !first) {
        const double nd = P.distinct ? S[S_XY2] : 0.0;
        if (!nest && nd > 0.0 && P.have_ry2) {
            const double num = 0.5 * S[S_RY2] + P.alpha * S[S_BRY];
            P.mu = fmax(fmin(P.mu, num / (0.5 * nd)), 0.0);
        }
        const double q = P.mu / P.L, th2 = P.theta * P.theta, bq = th2 - q;
        const double theta_n = 0.5 * (-bq + sqrt(bq * bq + 4.0 * th2));
        P.beta = P.theta * (1.0 - P.theta) / (th2 + theta_n);
        P.theta = theta_n;
        P.Y = P.YB;
        P.RY = P.RYB;
        P.distinct = 1;
        P.ex = 1;
        P.ry2_pending = 1;
        P.have_ry2 = 1;
    } else {
        P.Y = P.X;
        P.RY = P.RX;
        P.distinct = 0;
    }
    if (P.iters >= P.max_iter) {
        P.state = B_NOTCONV;
        P.need_grad = 0;
        P.ex = 0;
        return;
    }
    P.need_grad = 1;
    P.grad_evals++;
}

template <typename T>
__global__ __launch_bounds__(1024) void control_kernel(BatchProblem<T> *probs, int n,
                                                       int *running)
{
    int cnt = 0;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        BatchProblem<T> &P = probs[p];
        if (P.state == B_RUNNING)
            control_step(P);
        cnt += P.state == B_RUNNING ? 1 : 0;
    }
    __shared__ int sh[16];
    for (int off = 32; off > 0; off >>= 1)
        cnt += __shfl_down(cnt, off, 64);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w)
            s += sh[w];
        *running = s;
    }
}

}  // namespace

template <typename T>
hipError_t launch_control_batched(BatchProblem<T> *probs, int n, int *running, hipStream_t st)
{
    const int threads = std::min(1024, std::max(64, (n + 63) / 64 * 64));
    hipLaunchKernelGGL((control_kernel<T>), dim3(1), dim3(threads), 0, st, probs, n, running);
    return hipGetLastError();
}

template hipError_t launch_control_batched<float>(BatchProblem<float> *, int, int *, hipStream_t);
template hipError_t launch_control_batched<double>(BatchProblem<double> *, int, int *,
                                                   hipStream_t);

// ------------------------------------------------------------- host driver

namespace {

// Kernel families of a round, each with its own prefix table of block counts.
// The on-the-fly backprojector has one family per voxel depth (F_BP4,
// F_BP8) and the projector one per ray tile (6 widths x 4 block heights,
// from F_PJ), so that every problem runs its own tuned tiles, each family in
// a kernel compiled for that shape alone.
// Problems whose scan has a symmetry take the symmetric gather, one family
// per group (turns, mirror): F_BPS .. F_BPS + 4.
constexpr int PJ_FAMILY_WC[6] = {1, 2, 8, 16, 32, 64};
constexpr int PJ_FAMILY_TY[4] = {1, 2, 4, 8};
constexpr int N_PJ = 24;
constexpr int BPS_ROT[5] = {4, 4, 2, 2, 1}, BPS_MIR[5] = {1, 0, 1, 0, 1};
enum Family : int {
    F_BP4 = 0, F_BP8, F_BPS, F_SP = F_BPS + 5, F_VOX, F_TR, F_EX, F_PJ, F_COUNT = F_PJ + N_PJ
};
constexpr int BP_FAMILY_CZ[2] = {4, 8};

// Per-problem region: X, XB, YB, G, XT (N values each), RX, RXB, RYB (m
// each), the partial-sum slots and the finalised sums.
void region_layout(const tvreg_geometry *G, size_t (&vecN)[5], size_t (&vecM)[3], size_t &part,
                   size_t &sum, size_t &per)
{
    const size_t es = elem_size(G->prec);
    size_t off = 0;
    for (int i = 0; i < 5; ++i) {
        vecN[i] = off;
        off = align_up(off + es * (size_t)G->N, 256);
    }
    for (int i = 0; i < 3; ++i) {
        vecM[i] = off;
        off = align_up(off + es * (size_t)G->m, 256);
    }
    part = off;
    off = align_up(off + partial_bytes(G->pstride), 256);
    sum = off;
    off = align_up(off + sizeof(double) * S_COUNT, 256);
    per = off;
}

size_t batch_bytes(int n, const tvreg_geometry *const *geoms, std::vector<size_t> *base)
{
    const size_t ps = geoms[0]->prec == TVREG_F64 ? sizeof(BatchProblem<double>)
                                                  : sizeof(BatchProblem<float>);
    size_t off = align_up(ps * (size_t)n, 256);
    off = align_up(off + sizeof(int) * (size_t)F_COUNT * (n + 1), 256);
    off = align_up(off + 256, 256);  // running count
    for (int i = 0; i < n; ++i) {
        size_t vN[5], vM[3], part, sum, per;
        region_layout(geoms[i], vN, vM, part, sum, per);
        if (base)
            base->push_back(off);
        off += per;
    }
    return off;
}

// the projector family of a geometry's ray tile (the tuner's values)
int pj_family(const GeomDev &g)
{
    int a = 5, i = 2;  // 64 columns, 4 waves
    for (int k = 0; k < 6; ++k)
        if (PJ_FAMILY_WC[k] == g.pj_wc)
            a = k;
    for (int k = 0; k < 4; ++k)
        if (PJ_FAMILY_TY[k] == g.pj_ty)
            i = k;
    return F_PJ + 4 * a + i;
}

// Grouped launches run every problem with its geometry's tile shapes (and its
// stored transpose, when attached), except a backprojector depth of 16, which
// runs at 8: the grouped kernel at depth 16 needs 256 registers per lane, one
// wave per SIMD.
GeomDev batch_shapes(const GeomDev &g0)
{
    GeomDev g = g0;
    g.bp_cz = backproject_depth(g0) == 4 ? 4 : 8;
    return g;
}

int family_blocks(const tvreg_geometry *G, int f)
{
    const GeomDev g = batch_shapes(G->g);
    if (f >= F_PJ)
        return pj_family(g) == f ? project_blocks(g) : 0;
    const bool sym = !g.mat.present && backproject_symmetric(g);
    if (f >= F_BP4 && f <= F_BP8)
        return !g.mat.present && !sym && backproject_depth(g) == BP_FAMILY_CZ[f - F_BP4]
                   ? backproject_blocks(g)
                   : 0;
    if (f >= F_BPS && f < F_BPS + 5)
        return sym && g.sym_rot == BPS_ROT[f - F_BPS] && g.sym_mir == BPS_MIR[f - F_BPS]
                   ? backproject_sym_blocks(g)
                   : 0;
    switch (f) {
    case F_SP:
        return g.mat.present ? matrix_product_blocks(g) : 0;
    case F_VOX:
        return max_reduce_blocks_vol(g.nx, g.ny, g.nz);
    case F_TR:
        return companion_blocks(g);
    default:
        return elementwise_blocks(G->N) + elementwise_blocks(G->m);
    }
}

template <typename T>
tvreg_status batched_impl(int n, const tvreg_geometry *const *geoms, const void *const *b_dev,
                          const tvreg_solve_params *params, void *const *x_io, char *ws,
                          int poll, tvreg_solve_info *infos, hipStream_t st)
{
    std::vector<size_t> base;
    (void)batch_bytes(n, geoms, &base);
    const size_t ps = sizeof(BatchProblem<T>);
    BatchProblem<T> *dprobs = (BatchProblem<T> *)ws;
    int *doffs = (int *)(ws + align_up(ps * (size_t)n, 256));
    int *drunning =
        (int *)(ws + align_up(align_up(ps * (size_t)n, 256) +
                                  sizeof(int) * (size_t)F_COUNT * (n + 1),
                              256));

    // prefix tables of block counts, one per kernel family
    std::vector<int> offs((size_t)F_COUNT * (n + 1));
    int total[F_COUNT];
    for (int f = 0; f < F_COUNT; ++f) {
        int64_t acc = 0;
        for (int i = 0; i < n; ++i) {
            offs[(size_t)f * (n + 1) + i] = (int)acc;
            acc += family_blocks(geoms[i], f);
        }
        if (acc >= (int64_t(1) << 31))
            return fail(TVREG_EINVAL, "batch too large for one grouped launch");
        offs[(size_t)f * (n + 1) + n] = (int)acc;
        total[f] = (int)acc;
    }

    // start points and first gradients, one problem at a time
    std::vector<BatchProblem<T>> hp((size_t)n);
    for (int i = 0; i < n; ++i) {
        const tvreg_geometry *G = geoms[i];
        const tvreg_solve_params *p = params + i;
        size_t vN[5], vM[3], part, sum, per;
        region_layout(G, vN, vM, part, sum, per);
        char *r = ws + base[i];
        BatchProblem<T> &P = hp[i];
        memset(&P, 0, sizeof(P));
        P.g = batch_shapes(G->g);
        P.N = (int)G->N;
        P.m = (int)G->m;
        P.nb_vox = max_reduce_blocks_vol(G->g.nx, G->g.ny, G->g.nz);
        P.nb_proj = project_blocks(P.g);
        P.nb_ew = elementwise_blocks(G->m);
        P.pstride = G->pstride;
        P.X = (T *)(r + vN[0]);
        P.XB = (T *)(r + vN[1]);
        P.YB = (T *)(r + vN[2]);
        P.G = (T *)(r + vN[3]);
        P.XT = (T *)(r + vN[4]);
        P.RX = (T *)(r + vM[0]);
        P.RXB = (T *)(r + vM[1]);
        P.RYB = (T *)(r + vM[2]);
        P.Y = P.X;
        P.RY = P.RX;
        P.b = (const T *)b_dev[i];
        P.part = (double *)(r + part);
        P.sum = (double *)(r + sum);
        P.alpha = p->alpha;
        P.tau = p->tau;
        P.eps = p->eps;
        P.rho = p->rho_L;
        P.mu_bar = p->mu_bar;
        P.box = box_for<T>(p);
        if (!(P.box.lo <= P.box.hi))
            return fail(TVREG_EINVAL, "problem %d: box narrower than the storage precision", i);
        P.L = p->L_bar;
        P.phi = NAN;
        P.method = p->method;
        P.stop_mode = p->stop_mode;
        P.max_iter = p->max_iter;
        P.max_trials = p->max_trials;
        P.state = B_RUNNING;
        P.first = 1;
        P.grad_evals = 1;
        const GeomDev &g = P.g;
        TVR_HIP(launch_clip<T>(G->N, (const T *)x_io[i], P.X, P.box, st));
        TVR_HIP(launch_companion<T>(g, P.X, P.XT, st));
        TVR_HIP(launch_project<T>(g, P.X, P.XT, P.b, P.RX, nullptr, P.part, P.pstride, st,
                                  nullptr));
        TVR_HIP(launch_backproject<T>(g, P.RX, P.G, st));
        TVR_HIP(launch_tv<T>(g.nx, g.ny, g.nz, P.tau, P.alpha, P.X, nullptr, P.G, P.G, P.part,
                             P.pstride, st, nullptr));
        TVR_HIP(hipMemsetAsync(P.sum, 0, sizeof(double) * S_COUNT, st));
    }
    TVR_HIP(hipMemcpyAsync(dprobs, hp.data(), ps * (size_t)n, hipMemcpyHostToDevice, st));
    TVR_HIP(hipMemcpyAsync(doffs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice,
                           st));
    TVR_HIP(hipStreamSynchronize(st));  // host copies are read before they go out of scope

    // one round, captured on a private stream (kernel launches only)
    hipStream_t cs = nullptr;
    TVR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        hipGraph_t g = nullptr;
        hipGraphExec_t e = nullptr;
        ~StreamGuard()
        {
            if (e)
                (void)hipGraphExecDestroy(e);
            if (g)
                (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(s);
        }
    } guard{cs};
    auto fam = [&](int f) { return doffs + (size_t)f * (n + 1); };
    TVR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int f = F_BP4; f <= F_BP8; ++f)
        if (le == hipSuccess && total[f] > 0)
            le = launch_backproject_grouped<T>(dprobs, fam(f), n, total[f],
                                               BP_FAMILY_CZ[f - F_BP4], cs);
    for (int f = F_BPS; f < F_BPS + 5; ++f)
        if (le == hipSuccess && total[f] > 0)
            le = launch_backproject_sym_grouped<T>(dprobs, fam(f), n, total[f],
                                                   BPS_ROT[f - F_BPS], BPS_MIR[f - F_BPS], cs);
    if (le == hipSuccess && total[F_SP] > 0)
        le = launch_spmv_grouped<T>(dprobs, fam(F_SP), n, total[F_SP], cs);
    if (le == hipSuccess)
        le = launch_tv_grouped<T>(dprobs, fam(F_VOX), n, total[F_VOX], cs);
    if (le == hipSuccess)
        le = launch_trial_grouped<T>(dprobs, fam(F_VOX), n, total[F_VOX], cs);
    if (le == hipSuccess)
        le = launch_transpose_grouped<T>(dprobs, fam(F_TR), n, total[F_TR], cs);
    bool pj_buf = true;  // the walk's buffer-resource loads for every problem
    for (int i = 0; i < n; ++i)
        pj_buf = pj_buf && walk_buffer_ok(geoms[i]->g, sizeof(T));
    for (int f = F_PJ; f < F_COUNT; ++f)
        if (le == hipSuccess && total[f] > 0)
            le = launch_project_grouped<T>(dprobs, fam(f), n, total[f],
                                           PJ_FAMILY_WC[(f - F_PJ) / 4],
                                           PJ_FAMILY_TY[(f - F_PJ) % 4], pj_buf, cs);
    if (le == hipSuccess)
        le = launch_finalize_grouped<T>(dprobs, n, cs);
    if (le == hipSuccess)
        le = launch_control_batched<T>(dprobs, n, drunning, cs);
    if (le == hipSuccess)
        le = launch_extrapolate_grouped<T>(dprobs, fam(F_EX), n, total[F_EX], cs);
    const hipError_t ce = hipStreamEndCapture(cs, &guard.g);
    TVR_HIP(le);
    TVR_HIP(ce);
    TVR_HIP(hipGraphInstantiate(&guard.e, guard.g, nullptr, nullptr, 0));

    // every problem ends within max_iter * max_trials rounds
    int64_t max_rounds = 0;
    for (int i = 0; i < n; ++i)
        max_rounds = std::max(max_rounds, (int64_t)params[i].max_iter * params[i].max_trials);
    const int chunk = poll > 0 ? poll : 8;
    int running = n;
    for (int64_t r = 0; r < max_rounds && running > 0;) {
        for (int c = 0; c < chunk && r < max_rounds; ++c, ++r)
            TVR_HIP(hipGraphLaunch(guard.e, st));
        TVR_HIP(hipMemcpyAsync(&running, drunning, sizeof(int), hipMemcpyDeviceToHost, st));
        TVR_HIP(hipStreamSynchronize(st));
    }
    if (running > 0)
        return fail(TVREG_EDEVICE, "batched solve did not finish within its round bound");

    TVR_HIP(hipMemcpyAsync(hp.data(), dprobs, ps * (size_t)n, hipMemcpyDeviceToHost, st));
    TVR_HIP(hipStreamSynchronize(st));
    tvreg_status worst = TVREG_OK;
    for (int i = 0; i < n; ++i) {
        const BatchProblem<T> &P = hp[i];
        tvreg_solve_info &inf = infos[i];
        memset(&inf, 0, sizeof(inf));
        inf.iters = P.iters;
        inf.grad_evals = P.grad_evals;
        inf.func_evals = P.func_evals;
        inf.phi = P.phi;
        inf.gm_rel = P.gm0 > 0 ? P.gm / P.gm0 : 0.0;
        inf.gm_abs_over_N = P.gm / (double)P.N;
        inf.L = P.L;
        inf.mu = P.method == TVREG_UPN || P.method == TVREG_NESTEROV ? P.mu : 0.0;
        inf.stop_reason = P.state == B_CONVERGED ? TVREG_OK
                          : P.state == B_STALL   ? TVREG_ESTALL
                                                 : TVREG_ENOTCONV;
        if (inf.stop_reason == TVREG_ESTALL || (worst == TVREG_OK && inf.stop_reason != TVREG_OK))
            worst = (tvreg_status)inf.stop_reason;
        TVR_HIP(hipMemcpyAsync(x_io[i], P.X, sizeof(T) * (size_t)P.N, hipMemcpyDeviceToDevice,
                               st));
    }
    TVR_HIP(hipStreamSynchronize(st));
    return worst;
}

}  // namespace

}  // namespace tvr

using namespace tvr;

extern "C" size_t tvreg_solve_batched_workspace_bytes(int32_t n,
                                                      const tvreg_geometry *const *geoms)
{
    if (n < 1 || !geoms)
        return 0;
    for (int i = 0; i < n; ++i)
        if (!geoms[i] || geoms[i]->prec != geoms[0]->prec)
            return 0;
    return batch_bytes(n, geoms, nullptr);
}

extern "C" tvreg_status tvreg_solve_batched(int32_t n, const tvreg_geometry *const *geoms,
                                            const void *const *b_dev,
                                            const tvreg_solve_params *params,
                                            void *const *x_inout_dev, void *ws, size_t ws_bytes,
                                            int32_t poll_rounds, tvreg_solve_info *infos,
                                            void *stream)
{
    clear_error();
    if (n < 1 || !geoms || !b_dev || !params || !x_inout_dev || !infos)
        return fail(TVREG_EINVAL, "need n >= 1 and non-NULL arrays");
    for (int i = 0; i < n; ++i) {
        if (!geoms[i] || !b_dev[i] || !x_inout_dev[i])
            return fail(TVREG_EINVAL, "problem %d: NULL geometry or buffer", i);
        if (geoms[i]->prec != geoms[0]->prec || geoms[i]->device != geoms[0]->device)
            return fail(TVREG_EINVAL, "problem %d: precision or device differs from problem 0",
                        i);
        TVR_TRY(check_solve_params(params + i));
        if (params[i].method == TVREG_GPBB)
            return fail(TVREG_EINVAL, "problem %d: GPBB is not batched", i);
    }
    const size_t need = batch_bytes(n, geoms, nullptr);
    if (!ws || ws_bytes < need)
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed", need);
    DeviceGuard dg(geoms[0]->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", geoms[0]->device);
    hipStream_t st = (hipStream_t)stream;
    if (geoms[0]->prec == TVREG_F64)
        return batched_impl<double>(n, geoms, b_dev, params, x_inout_dev, (char *)ws, poll_rounds,
                                    infos, st);
    return batched_impl<float>(n, geoms, b_dev, params, x_inout_dev, (char *)ws, poll_rounds,
                               infos, st);
}
