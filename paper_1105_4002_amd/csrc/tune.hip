// Autotuner of the on-the-fly operators' tile shapes: the projector's ray
// tile per wavefront and waves per block, and the gather backprojector's
// voxels per thread along z.  Both operators visit the same rays and voxels
// in the same per-output order whatever the shape (a thread owns a ray, or
// a voxel column chunk), so the choice changes speed only; their control
// flow does not depend on the data, so zero-filled operands time them
// faithfully.
#include <algorithm>
#include <cmath>

#include "host.hpp"

using namespace tvr;

namespace {

constexpr int WC_SHAPES[6] = {1, 2, 8, 16, 32, 64};
constexpr int PJ_SHAPES[4] = {1, 2, 4, 8};
constexpr int BP_SHAPES[3] = {4, 8, 16};

bool valid_cols(int v) { return std::find(WC_SHAPES, WC_SHAPES + 6, v) != WC_SHAPES + 6; }
bool valid_waves(int v) { return std::find(PJ_SHAPES, PJ_SHAPES + 4, v) != PJ_SHAPES + 4; }
bool valid_depth(int v) { return std::find(BP_SHAPES, BP_SHAPES + 3, v) != BP_SHAPES + 3; }

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    }
};

// mean ms of `reps` launches of f after one warm-up launch
template <typename F>
tvreg_status time_launches(F f, int reps, hipStream_t st, Events &ev, double &ms)
{
    TVR_HIP(f());
    TVR_HIP(hipEventRecord(ev.a, st));
    for (int i = 0; i < reps; ++i)
        TVR_HIP(f());
    TVR_HIP(hipEventRecord(ev.b, st));
    TVR_HIP(hipEventSynchronize(ev.b));
    float t = 0.f;
    TVR_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
    ms = (double)t / reps;
    return TVREG_OK;
}

template <typename T>
tvreg_status tune_impl(tvreg_geometry *G, char *ws, int reps, tvreg_tuning *out, hipStream_t st)
{
    const size_t es = sizeof(T);
    const int64_t N = G->N, m = G->m;
    T *x = (T *)ws;
    T *xt = (T *)(ws + align_up(es * N, 256));
    T *xo = (T *)(ws + 2 * align_up(es * N, 256));
    T *b = (T *)(ws + 3 * align_up(es * N, 256));
    T *y = (T *)((char *)b + align_up(es * m, 256));
    double *part = (double *)((char *)y + align_up(es * m, 256));
    TVR_HIP(hipMemsetAsync(ws, 0, 3 * align_up(es * N, 256) + 2 * align_up(es * m, 256), st));

    Events ev;
    TVR_HIP(hipEventCreate(&ev.a));
    TVR_HIP(hipEventCreate(&ev.b));
    GeomDev g = G->g;
    g.mat = MatDev{};
    tvreg_tuning t{};
    double best = INFINITY;
    t.project_tile_cols = G->g.pj_wc;
    t.project_waves = G->g.pj_ty;
    for (int a = 0; a < 6; ++a) {
        for (int i = 0; i < 4; ++i) {
            g.pj_wc = WC_SHAPES[a];
            g.pj_ty = PJ_SHAPES[i];
            TVR_TRY(time_launches(
                [&] {
                    return launch_project<T>(g, x, xt, b, y, nullptr, part, G->pstride, st,
                                             nullptr);
                },
                reps, st, ev, t.project_ms[a][i]));
            if (t.project_ms[a][i] < best) {
                best = t.project_ms[a][i];
                t.project_tile_cols = WC_SHAPES[a];
                t.project_waves = PJ_SHAPES[i];
            }
        }
    }
    best = INFINITY;
    t.backproject_depth = G->g.bp_cz;
    for (int i = 0; i < 3; ++i) {
        g.bp_cz = BP_SHAPES[i];
        TVR_TRY(time_launches([&] { return launch_backproject<T>(g, y, xo, st); }, reps, st, ev,
                              t.backproject_ms[i]));
        if (t.backproject_ms[i] < best) {
            best = t.backproject_ms[i];
            t.backproject_depth = BP_SHAPES[i];
        }
    }
    G->g.pj_wc = t.project_tile_cols;
    G->g.pj_ty = t.project_waves;
    G->g.bp_cz = t.backproject_depth;
    if (out)
        *out = t;
    return TVREG_OK;
}

}  // namespace

extern "C" size_t tvreg_autotune_workspace_bytes(const tvreg_geometry *G)
{
    if (!G)
        return 0;
    const size_t es = elem_size(G->prec);
    return 3 * align_up(es * G->N, 256) + 2 * align_up(es * G->m, 256) +
           partial_bytes(G->pstride);
}

extern "C" tvreg_status tvreg_autotune(tvreg_geometry *G, void *ws, size_t ws_bytes, int32_t reps,
                                       tvreg_tuning *out, void *stream)
{
    clear_error();
    if (!G || !ws)
        return fail(TVREG_EINVAL, "NULL geometry or workspace");
    if (reps < 1 || reps > 1000)
        return fail(TVREG_EINVAL, "reps must be in [1, 1000], got %d", reps);
    if (ws_bytes < tvreg_autotune_workspace_bytes(G))
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed",
                    tvreg_autotune_workspace_bytes(G));
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    return G->prec == TVREG_F64 ? tune_impl<double>(G, (char *)ws, reps, out, st)
                                : tune_impl<float>(G, (char *)ws, reps, out, st);
}

extern "C" tvreg_status tvreg_get_tuning(const tvreg_geometry *G, tvreg_tuning *out)
{
    clear_error();
    if (!G || !out)
        return fail(TVREG_EINVAL, "NULL geometry or output");
    *out = tvreg_tuning{};
    out->project_tile_cols = G->g.pj_wc;
    out->project_waves = G->g.pj_ty;
    out->backproject_depth = G->g.bp_cz;
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_set_tuning(tvreg_geometry *G, const tvreg_tuning *t)
{
    clear_error();
    if (!G || !t)
        return fail(TVREG_EINVAL, "NULL geometry or tuning");
    if (!valid_cols(t->project_tile_cols))
        return fail(TVREG_EINVAL, "project_tile_cols must be 1, 2, 8, 16, 32 or 64, got %d",
                    t->project_tile_cols);
    if (!valid_waves(t->project_waves))
        return fail(TVREG_EINVAL, "project_waves must be 1, 2, 4 or 8, got %d", t->project_waves);
    if (!valid_depth(t->backproject_depth))
        return fail(TVREG_EINVAL, "backproject_depth must be 4, 8 or 16, got %d",
                    t->backproject_depth);
    G->g.pj_wc = t->project_tile_cols;
    G->g.pj_ty = t->project_waves;
    G->g.bp_cz = t->backproject_depth;
    return TVREG_OK;
}
