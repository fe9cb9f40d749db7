// Host side of the C ABI declared in include/tvreg.h: geometry tables,
// argument checks, workspace layout and the GP / GPBB / UPN drivers.
//
// The drivers keep every vector on the device and every scalar decision in
// double on the host: after each line-search trial the FP64 sums of the
// trial's kernels are read back (one stream synchronisation per trial) and
// the test of Alg. 2 or Alg. 1 is evaluated; the mu estimate (eq. 9), the
// theta root and beta of Alg. 3 follow from the same sums.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "host.hpp"

using namespace tvr;

namespace {
thread_local std::string g_err;
}  // namespace

tvreg_status tvr::fail(tvreg_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

void tvr::clear_error() { g_err.clear(); }

tvreg_status tvr::check_solve_params(const tvreg_solve_params *p)
{
    if (p->method != TVREG_GP && p->method != TVREG_GPBB && p->method != TVREG_UPN &&
        p->method != TVREG_NESTEROV)
        return fail(TVREG_EINVAL, "unknown method %d", (int)p->method);
    if (!(p->tau > 0) || !isfinite(p->tau) || !(p->alpha >= 0) || !isfinite(p->alpha))
        return fail(TVREG_EINVAL, "tau must be > 0 and alpha >= 0");
    if (!(p->eps >= 0) || p->max_iter < 1 || !(p->L_bar > 0) || !(p->rho_L > 1) ||
        p->max_trials < 1)
        return fail(TVREG_EINVAL, "need eps >= 0, max_iter >= 1, L_bar > 0, rho_L > 1, "
                                  "max_trials >= 1");
    if (p->stop_mode != 0 && p->stop_mode != 1)
        return fail(TVREG_EINVAL, "stop_mode must be 0 or 1");
    if (p->method == TVREG_GPBB &&
        (p->gpbb_K < 0 || p->gpbb_K > 16 || !(p->gpbb_beta0 > 0 && p->gpbb_beta0 < 1) ||
         !(p->gpbb_sigma >= 0)))
        return fail(TVREG_EINVAL, "GPBB needs 0 <= K <= 16, 0 < beta0 < 1, sigma >= 0");
    if (p->hist_len < 0)
        return fail(TVREG_EINVAL, "hist_len < 0");
    if (p->method == TVREG_NESTEROV &&
        (!isfinite(p->L_bar) || !(p->mu_bar >= 0) || !(p->mu_bar <= p->L_bar)))
        return fail(TVREG_EINVAL, "Nesterov's method needs a finite L_bar and 0 <= mu_bar <= L_bar");
    if (p->use_box != 0 && p->use_box != 1)
        return fail(TVREG_EINVAL, "use_box must be 0 or 1");
    if (p->use_box && !(p->lower < p->upper))
        return fail(TVREG_EINVAL, "the box needs lower < upper (got %g, %g)", p->lower, p->upper);
    return TVREG_OK;
}

tvr::Box tvr::box_of(const tvreg_solve_params *p)
{
    return p->use_box ? Box{p->lower, p->upper} : ORTHANT;
}

extern "C" const char *tvreg_last_error(void) { return g_err.c_str(); }

extern "C" const char *tvreg_version(void) { return "tvreg-gfx950 0.1.0"; }

// The symmetry group of a scan that a stored transpose uses (see MatDev):
// turns about z and the z mirror.  A circular cone scan qualifies when view
// v + V/4 (V/2) is view v turned by a quarter (half) turn, to 1e-12 in its
// direction cosines; the detector must be even in both directions, so that
// no ray runs inside a voxel face (the half-open cells are not symmetric
// under a turn or a mirror).  Quarter turns need a square volume of even
// side, half turns an even ny, the mirror an even nz.
static void scan_symmetry(const tvreg_geometry_desc &d, const double *angles, int &rot, int &mir)
{
    rot = 1;
    mir = 0;
    if (d.beam != TVREG_CONE || d.det_cols % 2 || d.det_rows % 2)
        return;
    const int V = d.n_views;
    auto turned = [&](int step, double ang) {  // view (v + step) % V = view v turned by ang
        const double ca = cos(ang), sa = sin(ang);
        for (int v = 0; v < V; ++v) {
            const double a = angles[v], b = angles[(v + step) % V];
            const double c = cos(a), s = sin(a);
            if (fabs(cos(b) - (c * ca - s * sa)) > 1e-12 || fabs(sin(b) - (c * sa + s * ca)) > 1e-12)
                return false;
        }
        return true;
    };
    if (d.nx == d.ny && d.nx % 2 == 0 && V % 4 == 0 && turned(V / 4, 0.5 * M_PI))
        rot = 4;
    else if (d.ny % 2 == 0 && V % 2 == 0 && turned(V / 2, M_PI))
        rot = 2;
    if (d.nz % 2 == 0)
        mir = 1;
}

extern "C" tvreg_status tvreg_create_geometry(const tvreg_geometry_desc *d,
                                              tvreg_precision precision, tvreg_geometry **out)
{
    g_err.clear();
    if (!d || !out)
        return fail(TVREG_EINVAL, "NULL descriptor or output pointer");
    *out = nullptr;
    if (precision != TVREG_F32_RED64 && precision != TVREG_F64)
        return fail(TVREG_EINVAL, "unknown precision %d", (int)precision);
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->n_views < 1 || d->det_cols < 1 ||
        d->det_rows < 1)
        return fail(TVREG_EINVAL, "sizes must be >= 1");
    const bool p3 = d->beam == TVREG_PARALLEL_3D;
    if (!p3 && !d->angles_rad)
        return fail(TVREG_EINVAL, "angles_rad is NULL");
    if (p3 && !d->view_dirs)
        return fail(TVREG_EINVAL, "view_dirs is NULL for a 3D parallel beam");
    if (!(d->pitch_u > 0) || !(d->pitch_v > 0))
        return fail(TVREG_EINVAL, "detector pitches must be > 0");
    const int64_t N = (int64_t)d->nx * d->ny * d->nz;
    const int64_t m = (int64_t)d->n_views * d->det_rows * d->det_cols;
    if (N >= (int64_t(1) << 31) || m >= (int64_t(1) << 31))
        return fail(TVREG_EINVAL, "volume or data larger than 2^31 entries");
    if (d->nx + d->ny + d->nz > (1 << 20))
        return fail(TVREG_EINVAL, "volume side too large");
    const double half_diag =
        0.5 * sqrt((double)d->nx * d->nx + (double)d->ny * d->ny + (double)d->nz * d->nz);
    if (d->beam == TVREG_CONE) {
        if (!(d->src_to_centre > half_diag) || !(d->src_to_det - d->src_to_centre > half_diag))
            return fail(TVREG_EINVAL,
                        "cone beam needs source and detector outside the volume's bounding "
                        "sphere (R=%g, SDD=%g, half diagonal %g)",
                        d->src_to_centre, d->src_to_det, half_diag);
    } else if (d->beam != TVREG_PARALLEL && !p3) {
        return fail(TVREG_EINVAL, "unknown beam %d", (int)d->beam);
    }
    for (int v = 0; v < d->n_views; ++v) {
        if (p3) {
            const double *q = d->view_dirs + 3 * (size_t)v;
            if (!isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2]) ||
                !(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] > 0.0))
                return fail(TVREG_EINVAL, "view direction %d is not finite and nonzero", v);
        } else if (!isfinite(d->angles_rad[v])) {
            return fail(TVREG_EINVAL, "angle %d is not finite", v);
        }
    }

    const bool cone = d->beam == TVREG_CONE;
    const int V = d->n_views, C = d->det_cols, Rw = d->det_rows;
    const double cu0 = 0.5 * (double)(C - 1), rv0 = 0.5 * (double)(Rw - 1);
    const double R = d->src_to_centre, SDD = d->src_to_det;

    std::vector<double2> cs(V);
    // the 3D beam forms its rays from per-view tables: one placeholder entry
    // in the column / row tables, which nothing reads for it
    std::vector<ColEntry> colt(p3 ? 1 : (size_t)V * C);
    std::vector<RowEntry> rowt(p3 ? 1 : Rw);
    std::vector<double> dn(cone ? (size_t)Rw * C : (size_t)V);
    std::vector<View3> v3t(p3 ? V : 1);
    for (int v = 0; p3 && v < V; ++v) {
        const double *q = d->view_dirs + 3 * (size_t)v;
        const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        View3 &e = v3t[v];
        e.dx = q[0] / nq;
        e.dy = q[1] / nq;
        e.dz = q[2] / nq;
        const double a = sqrt(e.dx * e.dx + e.dy * e.dy);  // |e_z x d|
        if (a > 0.0) {
            e.ux = -e.dy / a;
            e.uy = e.dx / a;
        } else {
            e.ux = 1.0;
            e.uy = 0.0;
        }
        e.uz = 0.0;
        // e_v = d x e_u
        e.vx = e.dy * e.uz - e.dz * e.uy;
        e.vy = e.dz * e.ux - e.dx * e.uz;
        e.vz = e.dx * e.uy - e.dy * e.ux;
        e.idx = e.dx != 0.0 ? 1.0 / e.dx : 0.0;
        e.idy = e.dy != 0.0 ? 1.0 / e.dy : 0.0;
        e.idz = e.dz != 0.0 ? 1.0 / e.dz : 0.0;
        cs[v] = make_double2(e.dx, e.dy);
        dn[v] = 1.0;  // |d|
    }
    for (int v = 0; !p3 && v < V; ++v) {
        const double c = cos(d->angles_rad[v]), s = sin(d->angles_rad[v]);
        cs[v] = make_double2(c, s);
        for (int col = 0; col < C; ++col) {
            const double u = ((double)col - cu0) * d->pitch_u;
            ColEntry &e = colt[(size_t)v * C + col];
            if (cone) {
                e.Sx = R * c;
                e.Sy = R * s;
                e.Dx = -SDD * c - u * s;
                e.Dy = -SDD * s + u * c;
            } else {
                e.Sx = -u * s;
                e.Sy = u * c;
                e.Dx = c;
                e.Dy = s;
            }
            e.invDx = e.Dx != 0.0 ? 1.0 / e.Dx : 0.0;
            e.invDy = e.Dy != 0.0 ? 1.0 / e.Dy : 0.0;
            e.ox = -e.Sx * e.invDx;
            e.oy = -e.Sy * e.invDy;
        }
        if (!cone)
            dn[v] = sqrt(c * c + s * s);
    }
    for (int row = 0; !p3 && row < Rw; ++row) {
        const double w = ((double)row - rv0) * d->pitch_v;
        RowEntry &e = rowt[row];
        e.Sz = cone ? 0.0 : w;
        e.Dz = cone ? w : 0.0;
        e.invDz = e.Dz != 0.0 ? 1.0 / e.Dz : 0.0;
        e.oz = -e.Sz * e.invDz;
        if (cone)
            for (int col = 0; col < C; ++col) {
                const double u = ((double)col - cu0) * d->pitch_u;
                dn[(size_t)row * C + col] = sqrt(SDD * SDD + u * u + w * w);
            }
    }

    tvreg_geometry *G = new (std::nothrow) tvreg_geometry();
    if (!G)
        return fail(TVREG_ENOMEM, "host allocation failed");
    G->desc = *d;
    if (p3) {
        G->angles.assign((size_t)V, 0.0);
        G->dirs.assign(d->view_dirs, d->view_dirs + 3 * (size_t)V);
        G->desc.view_dirs = G->dirs.data();
    } else {
        G->angles.assign(d->angles_rad, d->angles_rad + V);
        G->desc.view_dirs = nullptr;
    }
    G->desc.angles_rad = G->angles.data();
    G->prec = precision;
    G->N = N;
    G->m = m;
    if (hipGetDevice(&G->device) != hipSuccess) {
        delete G;
        return fail(TVREG_EDEVICE, "no HIP device");
    }
    const size_t o_cs = 0;
    const size_t o_col = align_up(o_cs + sizeof(double2) * V, 256);
    const size_t o_row = align_up(o_col + sizeof(ColEntry) * colt.size(), 256);
    const size_t o_dn = align_up(o_row + sizeof(RowEntry) * rowt.size(), 256);
    const size_t o_v3 = align_up(o_dn + sizeof(double) * dn.size(), 256);
    const size_t total = align_up(o_v3 + sizeof(View3) * v3t.size(), 256);
    char *base = nullptr;
    if (hipMalloc((void **)&base, total) != hipSuccess) {
        delete G;
        return fail(TVREG_ENOMEM, "device allocation of %zu bytes failed", total);
    }
    hipError_t e = hipMemcpy(base + o_cs, cs.data(), sizeof(double2) * V, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_col, colt.data(), sizeof(ColEntry) * colt.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_row, rowt.data(), sizeof(RowEntry) * rowt.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_dn, dn.data(), sizeof(double) * dn.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_v3, v3t.data(), sizeof(View3) * v3t.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete G;
        return fail(TVREG_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
    }
    G->dev_tables = base;
    GeomDev &g = G->g;
    g.nx = d->nx;
    g.ny = d->ny;
    g.nz = d->nz;
    g.nviews = V;
    g.cols = C;
    g.rows = Rw;
    g.cone = cone ? 1 : 0;
    g.pu = d->pitch_u;
    g.pv = d->pitch_v;
    g.ipu = 1.0 / d->pitch_u;
    g.ipv = 1.0 / d->pitch_v;
    g.R = R;
    g.SDD = SDD;
    g.cu0 = cu0;
    g.rv0 = rv0;
    g.hx = 0.5 * d->nx;
    g.hy = 0.5 * d->ny;
    g.hz = 0.5 * d->nz;
    g.cs = (const double2 *)(base + o_cs);
    g.col = (const ColEntry *)(base + o_col);
    g.row = (const RowEntry *)(base + o_row);
    g.dnorm = (const double *)(base + o_dn);
    g.beam3d = p3 ? 1 : 0;
    g.v3 = p3 ? (const View3 *)(base + o_v3) : nullptr;
    g.mat = MatDev{};
    g.pj_wc = default_tile_cols(Rw);
    g.pj_ty = PJ_TY_DEFAULT;
    g.bp_cz = BP_CZ_DEFAULT;
    g.flat_row = -1;
    for (int row = 0; cone && row < Rw; ++row)
        if (rowt[row].invDz == 0.0)
            g.flat_row = row;
    scan_symmetry(G->desc, G->angles.data(), g.sym_rot, g.sym_mir);
    // partial sums sized for every projector tile shape the tuner may pick
    G->pstride = std::max({project_blocks_max(g), max_reduce_blocks_vol(g.nx, g.ny, g.nz),
                           elementwise_blocks(N), elementwise_blocks(m)});
    *out = G;
    return TVREG_OK;
}

extern "C" void tvreg_destroy_geometry(tvreg_geometry *G)
{
    if (!G)
        return;
    DeviceGuard dg(G->device);
    (void)hipFree(G->dev_tables);
    delete G;
}

extern "C" tvreg_status tvreg_project(const tvreg_geometry *G, const void *x, void *y,
                                      void *stream)
{
    g_err.clear();
    if (!G || !x || !y)
        return fail(TVREG_EINVAL, "NULL geometry or buffer");
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    if (G->prec == TVREG_F64)
        TVR_HIP((launch_project<double>(G->g, (const double *)x, nullptr, nullptr, (double *)y,
                                        nullptr, nullptr, 0, st, nullptr)));
    else
        TVR_HIP((launch_project<float>(G->g, (const float *)x, nullptr, nullptr, (float *)y,
                                       nullptr, nullptr, 0, st, nullptr)));
    return TVREG_OK;
}

extern "C" size_t tvreg_project_workspace_bytes(const tvreg_geometry *G)
{
    return G ? elem_size(G->prec) * (size_t)G->N : 0;
}

extern "C" tvreg_status tvreg_project_ws(const tvreg_geometry *G, const void *x, void *y,
                                         void *ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    if (!G || !x || !y || !ws)
        return fail(TVREG_EINVAL, "NULL geometry or buffer");
    if (ws_bytes < tvreg_project_workspace_bytes(G))
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed",
                    tvreg_project_workspace_bytes(G));
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    if (G->prec == TVREG_F64) {
        TVR_HIP(launch_companion<double>(G->g, (const double *)x, (double *)ws, st));
        TVR_HIP((launch_project<double>(G->g, (const double *)x, (const double *)ws, nullptr,
                                        (double *)y, nullptr, nullptr, 0, st, nullptr)));
    } else {
        TVR_HIP(launch_companion<float>(G->g, (const float *)x, (float *)ws, st));
        TVR_HIP((launch_project<float>(G->g, (const float *)x, (const float *)ws, nullptr,
                                       (float *)y, nullptr, nullptr, 0, st, nullptr)));
    }
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_backproject(const tvreg_geometry *G, const void *r, void *x,
                                          void *stream)
{
    g_err.clear();
    if (!G || !r || !x)
        return fail(TVREG_EINVAL, "NULL geometry or buffer");
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    if (G->prec == TVREG_F64)
        TVR_HIP((launch_backproject<double>(G->g, (const double *)r, (double *)x, st)));
    else
        TVR_HIP((launch_backproject<float>(G->g, (const float *)r, (float *)x, st)));
    return TVREG_OK;
}


extern "C" size_t tvreg_tv_workspace_bytes(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1)
        return 0;
    return partial_bytes(max_reduce_blocks_vol(nx, ny, nz));
}

extern "C" tvreg_status tvreg_tv_grad(int32_t nx, int32_t ny, int32_t nz,
                                      tvreg_precision precision, double tau, const void *x,
                                      void *grad, double *tv_value, void *ws, size_t ws_bytes,
                                      void *stream)
{
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(TVREG_EINVAL, "sizes must be >= 1");
    if ((int64_t)nx * ny * nz >= (int64_t(1) << 31))
        return fail(TVREG_EINVAL, "volume larger than 2^31 entries");
    if (!x || (!grad && !tv_value))
        return fail(TVREG_EINVAL, "NULL input, or neither gradient nor value requested");
    if (!(tau > 0) || !isfinite(tau))
        return fail(TVREG_EINVAL, "tau must be positive and finite");
    if (precision != TVREG_F32_RED64 && precision != TVREG_F64)
        return fail(TVREG_EINVAL, "unknown precision %d", (int)precision);
    const int pstride = max_reduce_blocks_vol(nx, ny, nz);
    if (tv_value && (!ws || ws_bytes < partial_bytes(pstride)))
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed", partial_bytes(pstride));
    hipStream_t st = (hipStream_t)stream;
    double *part = tv_value ? (double *)ws : nullptr;
    int nb = 0;
    if (precision == TVREG_F64)
        TVR_HIP((launch_tv<double>(nx, ny, nz, tau, 1.0, (const double *)x, nullptr, nullptr,
                                   (double *)grad, part, pstride, st, &nb)));
    else
        TVR_HIP((launch_tv<float>(nx, ny, nz, tau, 1.0, (const float *)x, nullptr, nullptr,
                                  (float *)grad, part, pstride, st, &nb)));
    if (tv_value) {
        SlotList sl{};
        sl.n = 1;
        sl.slot[0] = S_TVY;
        sl.count[0] = nb;
        sl.dst[0] = tv_value;
        TVR_HIP(launch_finalize(sl, part, pstride, st));
    }
    return TVREG_OK;
}

// ------------------------------------------------ TV without an allocation
// Per-block FP64 partial sums of tvreg_tv_grad_noalloc, [S_COUNT][blocks],
// for at most NOALLOC_BLOCKS blocks of the TV grid.  Each device holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress reports for the current device (the array's
// name is a host-side stand-in there, not a device address).
namespace {
constexpr int NOALLOC_BLOCKS = 32768;  // 512^3 voxels: 8 x 128 x 32 blocks
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES];
}  // namespace

static __device__ __align__(256) double scratch[(size_t)S_COUNT * NOALLOC_BLOCKS];

// Device address of `scratch` on the current device, looked up once per device.
static tvreg_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(TVREG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(TVREG_EDEVICE, "device %d outside the %d the library tracks", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TVREG_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                        hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_tv_grad_noalloc(int32_t nx, int32_t ny, int32_t nz,
                                              tvreg_precision precision, double tau,
                                              const void *x, void *grad, double *tv_value,
                                              void *stream)
{
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(TVREG_EINVAL, "sizes must be >= 1");
    if ((int64_t)nx * ny * nz >= (int64_t(1) << 31))
        return fail(TVREG_EINVAL, "volume larger than 2^31 entries");
    if (!x || (!grad && !tv_value))
        return fail(TVREG_EINVAL, "NULL input, or neither gradient nor value requested");
    if (!(tau > 0) || !isfinite(tau))
        return fail(TVREG_EINVAL, "tau must be positive and finite");
    if (precision != TVREG_F32_RED64 && precision != TVREG_F64)
        return fail(TVREG_EINVAL, "unknown precision %d", (int)precision);
    const int pstride = max_reduce_blocks_vol(nx, ny, nz);
    if (pstride > NOALLOC_BLOCKS)
        return fail(TVREG_EINVAL,
                    "volume %d x %d x %d needs %d TV blocks; the no-allocation scratch holds "
                    "partial sums for at most %d (%zu bytes)",
                    nx, ny, nz, pstride, NOALLOC_BLOCKS, sizeof(scratch));
    double *part = nullptr;
    if (tv_value) {
        void *p = nullptr;
        const tvreg_status s = scratch_address(&p);
        if (s != TVREG_OK)
            return s;
        part = (double *)p;
    }
    hipStream_t st = (hipStream_t)stream;
    int nb = 0;
    if (precision == TVREG_F64)
        TVR_HIP((launch_tv<double>(nx, ny, nz, tau, 1.0, (const double *)x, nullptr, nullptr,
                                   (double *)grad, part, pstride, st, &nb)));
    else
        TVR_HIP((launch_tv<float>(nx, ny, nz, tau, 1.0, (const float *)x, nullptr, nullptr,
                                  (float *)grad, part, pstride, st, &nb)));
    if (tv_value) {
        SlotList sl{};
        sl.n = 1;
        sl.slot[0] = S_TVY;
        sl.count[0] = nb;
        sl.dst[0] = tv_value;
        TVR_HIP(launch_finalize(sl, part, pstride, st));
    }
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_tv_hessvec(int32_t nx, int32_t ny, int32_t nz,
                                         tvreg_precision precision, double tau, const void *y,
                                         const void *v, void *out, double *grad_dot, void *ws,
                                         size_t ws_bytes, void *stream)
{
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(TVREG_EINVAL, "sizes must be >= 1");
    if ((int64_t)nx * ny * nz >= (int64_t(1) << 31))
        return fail(TVREG_EINVAL, "volume larger than 2^31 entries");
    if (!y || !v || !out)
        return fail(TVREG_EINVAL, "NULL y, v or out");
    if (out == y || out == v)
        return fail(TVREG_EINVAL, "out must not alias y or v");
    if (!(tau > 0) || !isfinite(tau))
        return fail(TVREG_EINVAL, "tau must be positive and finite");
    if (precision != TVREG_F32_RED64 && precision != TVREG_F64)
        return fail(TVREG_EINVAL, "unknown precision %d", (int)precision);
    const int pstride = max_reduce_blocks_vol(nx, ny, nz);
    if (grad_dot && (!ws || ws_bytes < partial_bytes(pstride)))
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed", partial_bytes(pstride));
    hipStream_t st = (hipStream_t)stream;
    double *part = grad_dot ? (double *)ws : nullptr;
    int nb = 0;
    if (precision == TVREG_F64)
        TVR_HIP((launch_hessvec<double>(nx, ny, nz, tau, (const double *)y, (const double *)v,
                                        nullptr, nullptr, 0.0, 0.0, 1.0, (double *)out, part,
                                        pstride, st, &nb)));
    else
        TVR_HIP((launch_hessvec<float>(nx, ny, nz, tau, (const float *)y, (const float *)v,
                                       nullptr, nullptr, 0.0, 0.0, 1.0, (float *)out, part,
                                       pstride, st, &nb)));
    if (grad_dot) {
        SlotList sl{};
        sl.n = 1;
        sl.slot[0] = S_AD1;
        sl.count[0] = nb;
        sl.dst[0] = grad_dot;
        TVR_HIP(launch_finalize(sl, part, pstride, st));
    }
    return TVREG_OK;
}

// ------------------------------------------------------------------ solver

namespace {

struct Layout {
    size_t vecN[6], vecM[3], partials, total;  // vecN[5]: transposed copy
};

Layout solve_layout(const tvreg_geometry *G)
{
    Layout L{};
    const size_t es = elem_size(G->prec);
    size_t off = 0;
    for (int i = 0; i < 6; ++i) {
        L.vecN[i] = off;
        off = align_up(off + es * (size_t)G->N, 256);
    }
    for (int i = 0; i < 3; ++i) {
        L.vecM[i] = off;
        off = align_up(off + es * (size_t)G->m, 256);
    }
    L.partials = off;
    off = align_up(off + partial_bytes(G->pstride), 256);
    L.total = off;
    return L;
}

// Opt-in per-kernel timing of the solver's launches (HIP events on the
// solver's stream, resolved at the next synchronisation).
struct ProfTotals {
    std::mutex mu;
    bool on = false;
    int64_t count[TVREG_KERNEL_COUNT] = {};
    double ms[TVREG_KERNEL_COUNT] = {};
};
ProfTotals g_prof;

struct Runner {
    const tvreg_geometry *G;
    hipStream_t st;
    double *part;
    int pstride;
    HostScalars hs;     // the slots' sums, written by the finaliser straight to host memory
    SlotList pend;
    bool prof = false;
    struct Ev {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<Ev> evs;
    std::vector<hipEvent_t> pool;

    ~Runner()
    {
        for (auto &e : evs) {
            pool.push_back(e.a);
            pool.push_back(e.b);
        }
        for (hipEvent_t e : pool)
            (void)hipEventDestroy(e);
    }
    hipEvent_t ev()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    // runs launch() bracketed by events when profiling is on
    template <class F>
    hipError_t timed(int kid, F &&launch)
    {
        if (!prof)
            return launch();
        Ev e{kid, ev(), ev()};
        (void)hipEventRecord(e.a, st);
        hipError_t r = launch();
        (void)hipEventRecord(e.b, st);
        evs.push_back(e);
        return r;
    }
    void resolve()  // stream already synchronised
    {
        if (evs.empty())
            return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        for (auto &e : evs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
                g_prof.count[e.kid]++;
                g_prof.ms[e.kid] += ms;
            }
            pool.push_back(e.a);
            pool.push_back(e.b);
        }
        evs.clear();
    }

    void add(int slot, int count)
    {
        for (int i = 0; i < pend.n; ++i)
            if (pend.slot[i] == slot) {
                pend.count[i] = count;
                return;
            }
        pend.slot[pend.n] = slot;
        pend.count[pend.n] = count;
        pend.dst[pend.n] = hs.p + slot;
        pend.n++;
    }
    tvreg_status read()
    {
        // the finaliser writes the pending sums into the page-locked host
        // slots (no separate copy); they are read once the stream is done
        TVR_HIP(launch_finalize(pend, part, pstride, st));
        pend.n = 0;
        TVR_HIP(spin_sync(st, hs.done));
        resolve();
        return TVREG_OK;
    }
};

bool stop_test(const tvreg_solve_params *p, double gm, double gm0, int64_t N)
{
    if (p->stop_mode == 1)
        return gm / (double)N <= p->eps;
    return gm0 == 0.0 || gm <= p->eps * gm0;
}

void hist_put(double *h, int32_t len, int k, double v)
{
    if (h && k >= 0 && k < len)
        h[k] = v;
}

template <typename T>
struct Solver {
    const tvreg_geometry *G;
    const tvreg_solve_params *p;
    const T *b;
    Runner run;
    int nx, ny, nz;
    int64_t N, m;
    T *vN[5];
    T *vM[3];
    T *xt;  // the projector's companion copy of the volume being projected

    tvreg_status project(const T *x, T *out, const T *rref)
    {
        int nb = 0;
        TVR_HIP(run.timed(TVREG_KERNEL_TRANSPOSE,
                          [&] { return launch_companion<T>(G->g, x, xt, run.st); }));
        TVR_HIP(run.timed(TVREG_KERNEL_PROJECT, [&] {
            return launch_project<T>(G->g, x, xt, b, out, rref, run.part, run.pstride, run.st,
                                     &nb);
        }));
        run.add(S_R2, nb);
        if (rref)
            run.add(S_RD2, nb);
        return TVREG_OK;
    }
    // g = A^T r + alpha grad T(y); the slot of T(y) (GPBB's objective values
    // only) and, with xref, the Bregman terms
    tvreg_status gradient(const T *y, const T *ry, const T *xref, T *g)
    {
        TVR_HIP(run.timed(TVREG_KERNEL_BACKPROJECT,
                          [&] { return launch_backproject<T>(G->g, ry, g, run.st); }));
        int nb = 0;
        const bool value = p->method == TVREG_GPBB;
        TVR_HIP(run.timed(TVREG_KERNEL_TV, [&] {
            return launch_tv<T>(nx, ny, nz, p->tau, p->alpha, y, xref, g, g, run.part,
                                run.pstride, run.st, &nb, value);
        }));
        if (value)
            run.add(S_TVY, nb);
        if (xref) {
            run.add(S_BRY, nb);
            run.add(S_XY2, nb);
        }
        return TVREG_OK;
    }
    tvreg_status trial(const T *z, const T *g, double step, double gm_step, T *xb)
    {
        int nb = 0;
        TVR_HIP(run.timed(TVREG_KERNEL_TRIAL, [&] {
            return launch_trial<T>(nx, ny, nz, p->tau, z, g, step, gm_step, box_for<T>(p), xb,
                                   run.part, run.pstride, run.st, &nb);
        }));
        run.add(S_XD2, nb);
        run.add(S_GD, nb);
        run.add(S_TVB, nb);
        run.add(S_BRB, nb);
        if (gm_step > 0)
            run.add(S_GM2, nb);
        return TVREG_OK;
    }

    // GP (beta = 0), UPN, and Nesterov's method for given mu and L (UPN with
    // L and mu held: no line-search test, no eq. 9 estimate).
    tvreg_status gp_upn(T *x_io, tvreg_solve_info *info)
    {
        const bool nest = p->method == TVREG_NESTEROV;
        const bool upn = p->method == TVREG_UPN || nest;
        T *X = vN[0], *XB = vN[1], *Ybuf = vN[2], *Gv = vN[3];
        T *RX = vM[0], *RXB = vM[1], *RYbuf = vM[2];
        TVR_HIP(launch_clip<T>(N, x_io, X, box_for<T>(p), run.st));
        TVR_TRY(project(X, RX, nullptr));
        T *Y = X, *RY = RX;
        TVR_TRY(gradient(Y, RY, nullptr, Gv));
        info->grad_evals++;

        // Alg. 2 at y with the Bregman-form acceptance test
        auto bt = [&](double L0, double &L, double &xd2, double &phi_xb) -> tvreg_status {
            L = L0;
            for (int t = 0; t < p->max_trials; ++t) {
                TVR_TRY(trial(Y, Gv, 1.0 / L, 0.0, XB));
                TVR_TRY(project(XB, RXB, RY));
                TVR_TRY(run.read());
                info->func_evals++;
                xd2 = run.hs[S_XD2];
                const double lhs = 0.5 * run.hs[S_RD2] + p->alpha * run.hs[S_BRB];
                phi_xb = 0.5 * run.hs[S_R2] + p->alpha * run.hs[S_TVB];
                if (nest || !(lhs > 0.5 * L * xd2))
                    return TVREG_OK;
                if (t + 1 < p->max_trials)
                    L *= p->rho_L;
            }
            return TVREG_ESTALL;
        };

        double L = 0, xd2 = 0, phi_xb = 0;
        tvreg_status st = bt(p->L_bar, L, xd2, phi_xb);
        const double gm0 = L * sqrt(xd2);
        double gm = gm0;
        info->iters = 1;
        info->L = L;
        double mu = nest ? p->mu_bar : (p->mu_bar > 0 ? p->mu_bar : 0.25 * L);
        double theta = sqrt(mu / L);
        double phi_out = phi_xb;
        hist_put(p->hist_phi, p->hist_len, 0, phi_xb);
        hist_put(p->hist_gm, p->hist_len, 0, 1.0);
        hist_put(p->hist_L, p->hist_len, 0, L);
        const T *out = XB;
        if (st == TVREG_ESTALL) {
            out = X;
            phi_out = NAN;
        } else if (st < 0) {
            return st;
        } else if (stop_test(p, gm0, gm0, N)) {
            st = TVREG_OK;
        } else {
            st = TVREG_ENOTCONV;
            std::swap(X, XB);
            std::swap(RX, RXB);
            Y = X;
            RY = RX;
            out = X;
            bool have_ry2 = false;
            for (int k = 1; k < p->max_iter; ++k) {
                const bool distinct = Y != X;
                TVR_TRY(gradient(Y, RY, distinct ? X : nullptr, Gv));
                info->grad_evals++;
                const tvreg_status bs = bt(L, L, xd2, phi_xb);
                if (bs < 0)
                    return bs;
                gm = L * sqrt(xd2);
                info->iters = k + 1;
                info->L = L;
                hist_put(p->hist_phi, p->hist_len, k, phi_xb);
                hist_put(p->hist_gm, p->hist_len, k, gm0 > 0 ? gm / gm0 : 0.0);
                hist_put(p->hist_L, p->hist_len, k, L);
                if (bs == TVREG_ESTALL) {
                    st = TVREG_ESTALL;
                    out = X;  // last accepted point x^(k)
                    break;
                }
                phi_out = phi_xb;
                if (stop_test(p, gm, gm0, N)) {
                    st = TVREG_OK;
                    out = XB;
                    break;
                }
                double beta = 0.0;
                if (upn) {
                    // eq. 9 between x^(k) and y^(k), skipped where they coincide
                    const double nd = distinct ? run.hs[S_XY2] : 0.0;
                    if (!nest && nd > 0.0 && have_ry2) {
                        const double num = 0.5 * run.hs[S_RY2] + p->alpha * run.hs[S_BRY];
                        mu = fmax(fmin(mu, num / (0.5 * nd)), 0.0);
                    }
                    const double q = mu / L, th2 = theta * theta, bq = th2 - q;
                    const double theta_n = 0.5 * (-bq + sqrt(bq * bq + 4.0 * th2));
                    beta = theta * (1.0 - theta) / (th2 + theta_n);
                    theta = theta_n;
                    // y^(k+1) = x^(k+1) + beta (x^(k+1) - x^(k)), and its residual
                    int nb = 0;
                    TVR_HIP(run.timed(TVREG_KERNEL_EXTRAPOLATE, [&] {
                        return launch_extrapolate2<T>(N, XB, X, Ybuf, m, RXB, RX, RYbuf, beta,
                                                      run.part, run.pstride, run.st, &nb);
                    }));
                    run.add(S_RY2, nb);
                    have_ry2 = true;
                    std::swap(X, XB);
                    std::swap(RX, RXB);
                    Y = Ybuf;
                    RY = RYbuf;
                } else {
                    std::swap(X, XB);
                    std::swap(RX, RXB);
                    Y = X;
                    RY = RX;
                }
                out = X;
            }
        }
        info->gm_rel = gm0 > 0 ? gm / gm0 : 0.0;
        info->gm_abs_over_N = gm / (double)N;
        info->mu = upn ? mu : 0.0;
        info->phi = phi_out;
        info->stop_reason = st;
        if (out != x_io)
            TVR_HIP(hipMemcpyAsync(x_io, out, sizeof(T) * (size_t)N, hipMemcpyDeviceToDevice,
                                   run.st));
        TVR_HIP(hipStreamSynchronize(run.st));
        if (st == TVREG_ESTALL && isnan(info->phi)) {
            // the start point was never accepted: report phi there
            info->phi = NAN;
        }
        return st;
    }

    // GPBB, Alg. 1
    tvreg_status gpbb(T *x_io, tvreg_solve_info *info)
    {
        T *X = vN[0], *XB = vN[1], *XP = vN[2], *Gv = vN[3], *GP = vN[4];
        T *RX = vM[0], *RXB = vM[1];
        TVR_HIP(launch_clip<T>(N, x_io, X, box_for<T>(p), run.st));
        TVR_TRY(project(X, RX, nullptr));
        TVR_TRY(gradient(X, RX, nullptr, Gv));
        info->grad_evals++;
        TVR_TRY(run.read());
        double fk = 0.5 * run.hs[S_R2] + p->alpha * run.hs[S_TVY];
        const int K = p->gpbb_K;
        double fh[17];
        int nf = 0;
        double theta = 1.0, gm0 = 0.0, gm = 0.0;
        tvreg_status st = TVREG_ENOTCONV;
        for (int k = 0; k < p->max_iter; ++k) {
            for (int q = (nf < K + 1 ? nf : K); q > 0; --q)
                fh[q] = fh[q - 1];
            fh[0] = fk;
            if (nf < K + 1)
                nf++;
            if (k > 0) {
                // gradient at x^(k); the previous one is kept for the BB step
                std::swap(Gv, GP);
                TVR_TRY(gradient(X, RX, nullptr, Gv));
                info->grad_evals++;
                int nb = 0;
                TVR_HIP(launch_bb_dots<T>(N, X, XP, Gv, GP, run.part, run.pstride, run.st, &nb));
                run.add(S_SS, nb);
                run.add(S_SY, nb);
                TVR_TRY(run.read());
                const double ss = run.hs[S_SS], sy = run.hs[S_SY];
                if (sy > 0.0 && ss > 0.0 && isfinite(ss / sy))
                    theta = ss / sy;
            }
            double fhat = fh[0];
            for (int q = 1; q < nf; ++q)
                fhat = fmax(fhat, fh[q]);
            double beta = p->gpbb_beta0, fb = 0.0;
            bool ok = false, stop = false;
            for (int sq = 0; sq <= p->max_trials; ++sq) {
                TVR_TRY(trial(X, Gv, beta * theta, sq == 0 ? theta : 0.0, XB));
                TVR_TRY(project(XB, RXB, nullptr));
                TVR_TRY(run.read());
                if (sq == 0) {
                    gm = sqrt(run.hs[S_GM2]) / theta;
                    if (k == 0)
                        gm0 = gm;
                    info->iters = k;
                    info->L = 1.0 / theta;
                    hist_put(p->hist_gm, p->hist_len, k, gm0 > 0 ? gm / gm0 : 0.0);
                    hist_put(p->hist_L, p->hist_len, k, 1.0 / theta);
                    hist_put(p->hist_phi, p->hist_len, k, fk);
                    if (stop_test(p, gm, gm0, N)) {
                        stop = true;
                        break;
                    }
                }
                info->func_evals++;
                fb = 0.5 * run.hs[S_R2] + p->alpha * run.hs[S_TVB];
                const double gd = run.hs[S_GD];
                if (!(fb >= fhat - p->gpbb_sigma * gd)) {
                    ok = true;
                    break;
                }
                beta = beta * beta;
            }
            if (stop) {
                st = TVREG_OK;
                break;
            }
            if (!ok) {
                st = TVREG_ESTALL;
                break;
            }
            // x^(k+1) = xbar
            T *t = XP;
            XP = X;
            X = XB;
            XB = t;
            std::swap(RX, RXB);
            fk = fb;
            info->iters = k + 1;
        }
        info->gm_rel = gm0 > 0 ? gm / gm0 : 0.0;
        info->gm_abs_over_N = gm / (double)N;
        info->mu = 0.0;
        info->phi = fk;
        info->stop_reason = st;
        TVR_HIP(hipMemcpyAsync(x_io, X, sizeof(T) * (size_t)N, hipMemcpyDeviceToDevice, run.st));
        TVR_HIP(hipStreamSynchronize(run.st));
        return st;
    }
};

}  // namespace

extern "C" size_t tvreg_solve_workspace_bytes(const tvreg_geometry *G, tvreg_method)
{
    if (!G)
        return 0;
    return solve_layout(G).total;
}

extern "C" size_t tvreg_objective_workspace_bytes(const tvreg_geometry *G)
{
    if (!G)
        return 0;
    return align_up(elem_size(G->prec) * (size_t)G->m, 256) +
           align_up(elem_size(G->prec) * (size_t)G->N, 256) + partial_bytes(G->pstride) + 256;
}

template <typename T>
static tvreg_status objective_impl(const tvreg_geometry *G, const T *b, double alpha, double tau,
                                   const T *x, T *grad, double *phi, char *ws, hipStream_t st)
{
    T *r = (T *)ws;
    T *xt = (T *)(ws + align_up(sizeof(T) * (size_t)G->m, 256));
    double *part = (double *)((char *)xt + align_up(sizeof(T) * (size_t)G->N, 256));
    double *sc = (double *)((char *)part + partial_bytes(G->pstride));
    int nb1 = 0, nb2 = 0;
    TVR_HIP(launch_companion<T>(G->g, x, xt, st));
    TVR_HIP(launch_project<T>(G->g, x, xt, b, r, nullptr, part, G->pstride, st, &nb1));
    TVR_HIP(launch_backproject<T>(G->g, r, grad, st));
    TVR_HIP(launch_tv<T>(G->g.nx, G->g.ny, G->g.nz, tau, alpha, x, nullptr, grad, grad, part,
                         G->pstride, st, &nb2));
    SlotList sl{};
    sl.n = 2;
    sl.slot[0] = S_R2;
    sl.count[0] = nb1;
    sl.dst[0] = sc;
    sl.slot[1] = S_TVY;
    sl.count[1] = nb2;
    sl.dst[1] = sc + 1;
    TVR_HIP(launch_finalize(sl, part, G->pstride, st));
    TVR_HIP(launch_combine_phi(sc, sc + 1, alpha, phi, st));
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_objective_grad(const tvreg_geometry *G, const void *b,
                                             double alpha, double tau, const void *x, void *grad,
                                             double *phi, void *ws, size_t ws_bytes,
                                             void *stream)
{
    g_err.clear();
    if (!G || !b || !x || !grad || !phi)
        return fail(TVREG_EINVAL, "NULL geometry or buffer");
    if (!(tau > 0) || !isfinite(tau) || !isfinite(alpha) || alpha < 0)
        return fail(TVREG_EINVAL, "tau must be > 0 and alpha >= 0");
    if (!ws || ws_bytes < tvreg_objective_workspace_bytes(G))
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed",
                    tvreg_objective_workspace_bytes(G));
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    if (G->prec == TVREG_F64)
        return objective_impl<double>(G, (const double *)b, alpha, tau, (const double *)x,
                                      (double *)grad, phi, (char *)ws, st);
    return objective_impl<float>(G, (const float *)b, alpha, tau, (const float *)x, (float *)grad,
                                 phi, (char *)ws, st);
}

template <typename T>
static tvreg_status solve_impl(const tvreg_geometry *G, const T *b, const tvreg_solve_params *p,
                               T *x, char *ws, tvreg_solve_info *info, hipStream_t st)
{
    if (!(box_for<T>(p).lo <= box_for<T>(p).hi))
        return fail(TVREG_EINVAL, "box narrower than the storage precision");
    const Layout L = solve_layout(G);
    Solver<T> s{};
    s.G = G;
    s.p = p;
    s.b = b;
    s.nx = G->g.nx;
    s.ny = G->g.ny;
    s.nz = G->g.nz;
    s.N = G->N;
    s.m = G->m;
    for (int i = 0; i < 5; ++i)
        s.vN[i] = (T *)(ws + L.vecN[i]);
    s.xt = (T *)(ws + L.vecN[5]);
    for (int i = 0; i < 3; ++i)
        s.vM[i] = (T *)(ws + L.vecM[i]);
    s.run.G = G;
    s.run.st = st;
    s.run.part = (double *)(ws + L.partials);
    s.run.pstride = G->pstride;
    s.run.pend.n = 0;
    if (!s.run.hs.p)
        return fail(TVREG_ENOMEM, "page-locked host buffer of %d doubles", (int)S_COUNT);
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        s.run.prof = g_prof.on;
    }
    std::fill(s.run.hs.p, s.run.hs.p + S_COUNT, 0.0);
    const tvreg_status r = p->method == TVREG_GPBB ? s.gpbb(x, info) : s.gp_upn(x, info);
    if (s.run.prof && hipStreamSynchronize(st) == hipSuccess)
        s.run.resolve();
    return r;
}

extern "C" tvreg_status tvreg_solve(const tvreg_geometry *G, const void *b,
                                    const tvreg_solve_params *p, void *x, void *ws,
                                    size_t ws_bytes, tvreg_solve_info *info, void *stream)
{
    g_err.clear();
    if (!G || !b || !p || !x || !info)
        return fail(TVREG_EINVAL, "NULL argument");
    TVR_TRY(check_solve_params(p));
    if (!ws || ws_bytes < solve_layout(G).total)
        return fail(TVREG_ENOMEM, "workspace of %zu bytes needed", solve_layout(G).total);
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    memset(info, 0, sizeof(*info));
    hipStream_t st = (hipStream_t)stream;
    if (G->prec == TVREG_F64)
        return solve_impl<double>(G, (const double *)b, p, (double *)x, (char *)ws, info, st);
    return solve_impl<float>(G, (const float *)b, p, (float *)x, (char *)ws, info, st);
}

// ------------------------------------------------------ stored system matrix

namespace {

struct MatLayout {
    int64_t sv, ev;
    size_t off_v, w_v, cnt_v, val_v, idx_v, total;
};

// The cell of voxels a stored transpose keeps (see MatDev): one cell of the
// symmetry group the geometry uses (scan_symmetry), when the packed ray key
// of the layout fits 31 bits; otherwise every voxel.
MatDev mat_cell(const tvreg_geometry *G)
{
    const tvreg_geometry_desc &d = G->desc;
    MatDev M{};
    M.rot = 1;
    M.mx = d.nx;
    M.my = d.ny;
    M.mz = d.nz;
    auto bits = [](int n) {
        int b = 0;
        while ((1 << b) < n)
            ++b;
        return b;
    };
    const int kc = bits(d.det_cols), kr = bits(d.det_rows), kv = bits(d.n_views);
    if ((G->g.sym_rot <= 1 && !G->g.sym_mir) || kc + kr + kv > 31)
        return M;
    if (G->g.sym_rot == 4) {
        M.rot = 4;
        M.mx = d.nx / 2;
        M.my = d.ny / 2;
    } else if (G->g.sym_rot == 2) {
        M.rot = 2;
        M.my = d.ny / 2;
    }
    if (G->g.sym_mir) {
        M.mir = 1;
        M.mz = d.nz / 2;
    }
    M.kc = kc;
    M.kr = kr;
    return M;
}

int mat_order(const MatDev &M) { return M.rot * (M.mir ? 2 : 1); }

// fixed part (slice table and counts), then the entries once counted
MatLayout mat_layout(const tvreg_geometry *G, int64_t ev)
{
    const MatDev C = mat_cell(G);
    MatLayout L{};
    L.sv = mat_slices(C.mx, C.my, C.mz);
    L.ev = ev;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.off_v = take(sizeof(int64_t) * (size_t)L.sv);
    L.w_v = take(sizeof(int32_t) * (size_t)L.sv);
    L.cnt_v = take(sizeof(int32_t) * (size_t)C.mx * C.my * C.mz);
    L.val_v = take(elem_size(G->prec) * (size_t)ev);
    L.idx_v = take(sizeof(int32_t) * (size_t)ev);
    L.total = off;
    return L;
}

// counts and slice widths into the given buffers, then the slice offsets
// (host) and the entry total (with padding)
tvreg_status count_entries(const tvreg_geometry *G, int32_t *cnt_v, int32_t *w_v, hipStream_t st,
                           std::vector<int64_t> &off_v, int64_t &ev, int64_t *nnz)
{
    GeomDev g = G->g;
    g.mat = mat_cell(G);
    const int64_t sv = mat_slices(g.mat.mx, g.mat.my, g.mat.mz);
    const size_t ncell = (size_t)g.mat.mx * g.mat.my * g.mat.mz;
    TVR_HIP(launch_matrix_count(g, cnt_v, st));
    TVR_HIP(launch_slice_widths(g, cnt_v, w_v, st));
    std::vector<int32_t> wv((size_t)sv);
    TVR_HIP(hipMemcpyAsync(wv.data(), w_v, sizeof(int32_t) * wv.size(), hipMemcpyDeviceToHost, st));
    std::vector<int32_t> cv;
    if (nnz) {
        cv.resize(ncell);
        TVR_HIP(hipMemcpyAsync(cv.data(), cnt_v, sizeof(int32_t) * cv.size(),
                               hipMemcpyDeviceToHost, st));
    }
    TVR_HIP(hipStreamSynchronize(st));
    off_v.resize((size_t)sv);
    ev = 0;
    for (int64_t s = 0; s < sv; ++s) {
        off_v[s] = ev;
        ev += 64 * (int64_t)wv[s];
    }
    if (nnz) {
        int64_t t = 0;
        for (int32_t c : cv)
            t += c;
        *nnz = t * mat_order(g.mat);  // every stored entry stands for its images
    }
    return TVREG_OK;
}

}  // namespace

extern "C" size_t tvreg_matrix_scratch_bytes(const tvreg_geometry *G)
{
    if (!G)
        return 0;
    return mat_layout(G, 0).val_v;  // the fixed part: slice table and counts
}

extern "C" tvreg_status tvreg_matrix_plan(const tvreg_geometry *G, void *scratch,
                                          size_t scratch_bytes, size_t *matrix_bytes,
                                          int64_t *nnz, void *stream)
{
    g_err.clear();
    if (!G || !matrix_bytes)
        return fail(TVREG_EINVAL, "NULL geometry or output");
    const MatLayout L0 = mat_layout(G, 0);
    if (!scratch || scratch_bytes < L0.val_v)
        return fail(TVREG_ENOMEM, "scratch of %zu bytes needed", L0.val_v);
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    char *b = (char *)scratch;
    std::vector<int64_t> off_v;
    int64_t ev = 0;
    TVR_TRY(count_entries(G, (int32_t *)(b + L0.cnt_v), (int32_t *)(b + L0.w_v),
                          (hipStream_t)stream, off_v, ev, nnz));
    *matrix_bytes = mat_layout(G, ev).total;
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_matrix_attach(tvreg_geometry *G, void *matrix, size_t matrix_bytes,
                                            void *stream)
{
    g_err.clear();
    if (!G || !matrix)
        return fail(TVREG_EINVAL, "NULL geometry or matrix buffer");
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    const MatLayout L0 = mat_layout(G, 0);
    if (matrix_bytes < L0.val_v)
        return fail(TVREG_ENOMEM, "matrix buffer smaller than its fixed part (%zu bytes)",
                    L0.val_v);
    char *b = (char *)matrix;
    std::vector<int64_t> off_v;
    int64_t ev = 0;
    TVR_TRY(count_entries(G, (int32_t *)(b + L0.cnt_v), (int32_t *)(b + L0.w_v), st, off_v, ev,
                          nullptr));
    const MatLayout L = mat_layout(G, ev);
    if (matrix_bytes < L.total)
        return fail(TVREG_ENOMEM, "matrix of %zu bytes needed", L.total);
    TVR_HIP(hipMemcpyAsync(b + L.off_v, off_v.data(), sizeof(int64_t) * off_v.size(),
                           hipMemcpyHostToDevice, st));
    MatDev M = mat_cell(G);
    M.present = 1;
    M.sv = L.sv;
    M.off_v = (const int64_t *)(b + L.off_v);
    M.w_v = (const int32_t *)(b + L.w_v);
    M.cnt_v = (const int32_t *)(b + L.cnt_v);
    M.val_v = b + L.val_v;
    M.idx_v = (const int32_t *)(b + L.idx_v);
    GeomDev g = G->g;
    g.mat = M;
    if (G->prec == TVREG_F64)
        TVR_HIP(launch_matrix_fill<double>(g, (double *)(b + L.val_v), (int32_t *)(b + L.idx_v),
                                           st));
    else
        TVR_HIP(launch_matrix_fill<float>(g, (float *)(b + L.val_v), (int32_t *)(b + L.idx_v),
                                          st));
    TVR_HIP(hipStreamSynchronize(st));
    G->g.mat = M;
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_matrix_detach(tvreg_geometry *G)
{
    g_err.clear();
    if (!G)
        return fail(TVREG_EINVAL, "NULL geometry");
    G->g.mat = MatDev{};
    return TVREG_OK;
}

extern "C" tvreg_status tvreg_set_symmetry(tvreg_geometry *G, int32_t use)
{
    g_err.clear();
    if (!G || (use != 0 && use != 1))
        return fail(TVREG_EINVAL, "NULL geometry or use not 0 / 1");
    if (G->g.mat.present)
        return fail(TVREG_EINVAL, "detach the stored transpose first");
    G->sym_off = use ? 0 : 1;
    int rot = 1, mir = 0;
    if (use)
        scan_symmetry(G->desc, G->angles.data(), rot, mir);
    G->g.sym_rot = rot;
    G->g.sym_mir = mir;
    return TVREG_OK;
}

extern "C" int32_t tvreg_matrix_symmetry(const tvreg_geometry *G)
{
    if (!G)
        return 0;
    return mat_order(G->g.mat.present ? G->g.mat : mat_cell(G));
}

extern "C" void tvreg_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
}

extern "C" void tvreg_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (int k = 0; k < TVREG_KERNEL_COUNT; ++k) {
        g_prof.count[k] = 0;
        g_prof.ms[k] = 0.0;
    }
}

extern "C" tvreg_status tvreg_profile_get(int32_t kernel, int64_t *count, double *total_ms)
{
    if (kernel < 0 || kernel >= TVREG_KERNEL_COUNT || !count || !total_ms)
        return fail(TVREG_EINVAL, "bad kernel id or NULL output");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    *count = g_prof.count[kernel];
    *total_ms = g_prof.ms[kernel];
    return TVREG_OK;
}
