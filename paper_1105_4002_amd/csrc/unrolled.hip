// Differentiated form: K unrolled UPN steps (Alg. 3 with BT, Alg. 2, and the
// mu estimate of eq. 9) from x^(0) = 0 and the reverse-mode gradient of a
// loss of x^(K) with respect to alpha and b.
//
// The forward pass records every scalar decision (L_j, mu_j and the branch
// of its min, theta_j, beta_j, and eq. 9's numerator parts) and keeps
// (x^(c), y^(c)) every `ckpt` steps.  The reverse pass walks the segments
// backwards: it recomputes a segment's iterates from its checkpoint with the
// same kernels and the recorded L_j and beta_j (bit-identical to the forward
// pass), then applies the adjoint of each step:
//   x^(j+1) = P_Q(y^(j) - (A^T (A y^(j) - b) + alpha grad T(y^(j))) / L_j)
//   y^(j+1) = x^(j+1) + beta_j (x^(j+1) - x^(j))
// with the L_j held fixed, the mask [x^(j+1) > 0] for P_Q, A^T A and the TV
// Hessian for the step's Jacobian, the root formula of theta for the
// schedule, and the eq. 9 quotient on the steps where its branch of the min
// was taken.  Scalars (the adjoints of alpha, beta, theta, mu) are FP64 on
// the host; vectors are T on the device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "host.hpp"

namespace tvr {

namespace {

constexpr int32_t TAPE_MAGIC = 0x7476756e;  // "tvun"

struct TapeHeader {
    int32_t magic, prec, K, ckpt, status, pad;
    int64_t N, m;
    double alpha, tau;
};

struct StepRec {
    double L, mu, theta, beta, M, B, D;
    int32_t state, pad;  // 3: step 0, 0: mu carried, 1: eq. 9 taken, 2: clamped to 0
};

struct TapeLayout {
    size_t header, recs, ck, fwd, seg, adj, part, sums, total;
};

int n_ckpt(int K, int ckpt) { return (K + ckpt - 1) / ckpt; }

TapeLayout tape_layout(const tvreg_geometry *G, int K, int ckpt)
{
    const size_t es = elem_size(G->prec);
    const size_t vN = align_up(es * (size_t)G->N, 256), vM = align_up(es * (size_t)G->m, 256);
    TapeLayout L{};
    size_t off = 0;
    L.header = off;
    off = align_up(off + sizeof(TapeHeader), 256);
    L.recs = off;
    off = align_up(off + sizeof(StepRec) * (size_t)(K + 1), 256);
    L.ck = off;
    off += vN * 2 * (size_t)n_ckpt(K, ckpt);
    L.fwd = off;  // X, XN, Y, YN, G, XT, then RX, RXB, RY
    off += 6 * vN + 3 * vM;
    L.seg = off;  // ckpt x's and ckpt - 1 y's beyond the checkpoint
    off += (size_t)(2 * ckpt) * vN;
    L.adj = off;  // XBN, XBC, YBN, YBC, ZB, W, DV, then P
    off += 7 * vN + vM;
    L.part = off;
    off = align_up(off + partial_bytes(G->pstride), 256);
    L.sums = off;
    off = align_up(off + sizeof(double) * S_COUNT, 256);
    L.total = off;
    return L;
}

template <typename T>
struct Unroller {
    const tvreg_geometry *G;
    const T *b;
    double alpha, tau;
    int K, ckpt;
    hipStream_t st;
    char *ws;
    TapeLayout lay;
    int64_t N, m;
    double *part, *dsum;
    HostScalars hs;  // host copy of the sums
    SlotList pend;

    T *vecN(size_t base, int i) const
    {
        return (T *)(ws + base + (size_t)i * align_up(sizeof(T) * (size_t)N, 256));
    }
    T *ckx(int c) const { return vecN(lay.ck, 2 * c); }
    T *cky(int c) const { return vecN(lay.ck, 2 * c + 1); }
    T *fwdN(int i) const { return vecN(lay.fwd, i); }
    T *fwdM(int i) const
    {
        return (T *)(ws + lay.fwd + 6 * align_up(sizeof(T) * (size_t)N, 256) +
                     (size_t)i * align_up(sizeof(T) * (size_t)m, 256));
    }
    T *segN(int i) const { return vecN(lay.seg, i); }
    T *adjN(int i) const { return vecN(lay.adj, i); }
    T *adjM() const { return (T *)(ws + lay.adj + 7 * align_up(sizeof(T) * (size_t)N, 256)); }

    void add(int slot, int count)
    {
        pend.slot[pend.n] = slot;
        pend.count[pend.n] = count;
        pend.dst[pend.n] = dsum + slot;
        pend.n++;
    }
    tvreg_status read()
    {
        TVR_HIP(launch_finalize(pend, part, G->pstride, st));
        pend.n = 0;
        TVR_HIP(hipMemcpyAsync(hs.p, dsum, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st));
        TVR_HIP(spin_sync(st, hs.done));
        return TVREG_OK;
    }

    // out = A x (- b), with the companion copy the projector reads
    tvreg_status project(const T *x, const T *bb, T *out, const T *rref, int *nb)
    {
        const GeomDev &g = G->g;
        TVR_HIP(launch_companion<T>(g, x, fwdN(5), st));
        TVR_HIP(launch_project<T>(g, x, fwdN(5), bb, out, rref, part, G->pstride, st, nb));
        return TVREG_OK;
    }
    // G = A^T (A y - b) + alpha grad T(y), the residual left in RY
    tvreg_status gradient(const T *y, const T *xref, T *RY, T *Gv, bool sums)
    {
        const GeomDev &g = G->g;
        int nbp = 0, nbt = 0;
        TVR_TRY(project(y, b, RY, sums ? xref_r : nullptr, &nbp));
        TVR_HIP(launch_backproject<T>(g, RY, Gv, st));
        TVR_HIP(launch_tv<T>(g.nx, g.ny, g.nz, tau, alpha, y, sums ? xref : nullptr, Gv, Gv,
                             sums ? part : nullptr, G->pstride, st, &nbt));
        if (sums) {
            add(S_RD2, nbp);
            add(S_BRY, nbt);
            add(S_XY2, nbt);
        }
        return TVREG_OK;
    }
    const T *xref_r = nullptr;  // residual of x^(j) for the eq. 9 sums

    // y^(j+1) from x^(j+1), x^(j) (a copy after step 0, where beta is not defined)
    tvreg_status advance_y(int j, double beta, const T *xn, const T *xo, T *yn)
    {
        if (j == 0) {
            TVR_HIP(hipMemcpyAsync(yn, xn, sizeof(T) * (size_t)N, hipMemcpyDeviceToDevice, st));
            return TVREG_OK;
        }
        TVR_HIP(launch_extrapolate<T>(N, beta, xn, xo, yn, nullptr, 0, st, nullptr));
        return TVREG_OK;
    }

    tvreg_status forward(const double *L_replay, double *L_out, T *xK, StepRec *rec,
                         const tvreg_solve_params *p, int *stall)
    {
        const GeomDev &g = G->g;
        T *X = fwdN(0), *XN = fwdN(1), *Y = fwdN(2), *YN = fwdN(3), *Gv = fwdN(4);
        T *RX = fwdM(0), *RXB = fwdM(1), *RY = fwdM(2);
        TVR_HIP(launch_lincomb<T>(N, nullptr, 0.0, nullptr, 0.0, nullptr, X, st));
        TVR_HIP(launch_lincomb<T>(N, nullptr, 0.0, nullptr, 0.0, nullptr, Y, st));
        double L = p->L_bar, theta = 0.0, mu = 0.0;
        *stall = 0;
        for (int j = 0; j < K; ++j) {
            if (j % ckpt == 0) {
                TVR_HIP(hipMemcpyAsync(ckx(j / ckpt), X, sizeof(T) * (size_t)N,
                                       hipMemcpyDeviceToDevice, st));
                TVR_HIP(hipMemcpyAsync(cky(j / ckpt), Y, sizeof(T) * (size_t)N,
                                       hipMemcpyDeviceToDevice, st));
            }
            // gradient at y^(j); for j >= 1 also the parts of eq. 9 between x^(j) and y^(j)
            xref_r = RX;
            TVR_TRY(gradient(Y, X, RY, Gv, j >= 1));
            double nd = 0.0, rd2 = 0.0, bry = 0.0;
            if (j >= 1) {
                TVR_TRY(read());
                nd = hs[S_XY2];
                rd2 = hs[S_RD2];
                bry = hs[S_BRY];
            }
            // step: BT (Alg. 2, Bregman form of its test) or the replayed L_j
            if (L_replay)
                L = L_replay[j];
            for (int t = 0;; ++t) {
                int nbt = 0, nbp = 0;
                TVR_HIP(launch_trial<T>(g.nx, g.ny, g.nz, tau, Y, Gv, 1.0 / L, 0.0, ORTHANT, XN,
                                        part, G->pstride, st, &nbt));
                TVR_TRY(project(XN, b, RXB, RY, &nbp));
                if (L_replay)
                    break;
                add(S_XD2, nbt);
                add(S_BRB, nbt);
                add(S_RD2, nbp);
                TVR_TRY(read());
                const double lhs = 0.5 * hs[S_RD2] + alpha * hs[S_BRB];
                if (!(lhs > 0.5 * L * hs[S_XD2]))
                    break;
                if (t + 1 >= p->max_trials) {
                    *stall = 1;
                    return TVREG_OK;
                }
                L *= p->rho_L;
            }
            StepRec &r = rec[j];
            r.L = L;
            if (L_out)
                L_out[j] = L;
            if (j == 0) {
                mu = p->mu_bar > 0.0 ? p->mu_bar : 0.25 * L;
                r.mu = mu;
                r.theta = 0.0;
                r.beta = 0.0;
                r.state = 3;
                theta = sqrt(mu / L);
                rec[1].theta = theta;
            } else {
                r.state = 0;
                if (nd > 0.0) {
                    r.B = bry;
                    r.D = 0.5 * nd;
                    r.M = (0.5 * rd2 + alpha * bry) / r.D;
                    if (r.M < mu) {
                        r.state = r.M >= 0.0 ? 1 : 2;
                        mu = r.M >= 0.0 ? r.M : 0.0;
                    }
                }
                r.mu = mu;
                const double q = mu / L, th2 = theta * theta, bq = th2 - q;
                const double tn = 0.5 * (-bq + sqrt(bq * bq + 4.0 * th2));
                r.beta = theta * (1.0 - theta) / (th2 + tn);
                theta = tn;
                rec[j + 1].theta = theta;
            }
            if (j + 1 < K)
                TVR_TRY(advance_y(j, r.beta, XN, X, YN));
            std::swap(X, XN);
            std::swap(RX, RXB);
            std::swap(Y, YN);
        }
        TVR_HIP(hipMemcpyAsync(xK, X, sizeof(T) * (size_t)N, hipMemcpyDeviceToDevice, st));
        return TVREG_OK;
    }

    // iterates x^(c..e) and y^(c..e-1) of one segment, from its checkpoint
    tvreg_status recompute(int c, int e, const StepRec *rec, std::vector<T *> &xs,
                           std::vector<T *> &ys)
    {
        const GeomDev &g = G->g;
        T *Gv = fwdN(4), *RY = fwdM(2);
        xs.assign(e - c + 1, nullptr);
        ys.assign(e - c, nullptr);
        xs[0] = ckx(c / ckpt);
        ys[0] = cky(c / ckpt);
        for (int j = c; j < e; ++j) {
            const int i = j - c;
            xs[i + 1] = segN(2 * i);
            TVR_TRY(gradient(ys[i], nullptr, RY, Gv, false));
            TVR_HIP(launch_trial<T>(g.nx, g.ny, g.nz, tau, ys[i], Gv, 1.0 / rec[j].L, 0.0,
                                    ORTHANT, xs[i + 1], part, G->pstride, st, nullptr));
            if (j + 1 < e) {
                ys[i + 1] = segN(2 * i + 1);
                TVR_TRY(advance_y(j, rec[j].beta, xs[i + 1], xs[i], ys[i + 1]));
            }
        }
        return TVREG_OK;
    }

    tvreg_status backward(const StepRec *rec, const T *xK_bar, T *b_bar, double *dl_dlogalpha)
    {
        const GeomDev &g = G->g;
        T *XBN = adjN(0), *XBC = adjN(1), *YBN = adjN(2), *YBC = adjN(3);
        T *ZB = adjN(4), *W = adjN(5), *DV = adjN(6), *P = adjM();
        TVR_HIP(hipMemcpyAsync(XBN, xK_bar, sizeof(T) * (size_t)N, hipMemcpyDeviceToDevice, st));
        for (T *v : {XBC, YBN, YBC})
            TVR_HIP(launch_lincomb<T>(N, nullptr, 0.0, nullptr, 0.0, nullptr, v, st));
        TVR_HIP(launch_lincomb<T>(m, nullptr, 0.0, nullptr, 0.0, nullptr, b_bar, st));
        std::vector<double> theta_bar(K + 2, 0.0), mu_bar(K + 1, 0.0);
        double abar = 0.0;
        std::vector<T *> xs, ys;
        for (int c = (n_ckpt(K, ckpt) - 1) * ckpt; c >= 0; c -= ckpt) {
            const int e = std::min(c + ckpt, K);
            TVR_TRY(recompute(c, e, rec, xs, ys));
            for (int j = e - 1; j >= c; --j) {
                const T *xj = xs[j - c], *xn = xs[j - c + 1], *yj = ys[j - c];
                const StepRec &r = rec[j];
                const double Lj = r.L;
                if (j >= 1 && j + 1 < K) {
                    // y^(j+1) = x^(j+1) + beta_j (x^(j+1) - x^(j))
                    int nb = 0;
                    TVR_HIP(launch_adj_extrap<T>(N, r.beta, YBN, xn, xj, XBN, XBC, part,
                                                 G->pstride, st, &nb));
                    add(S_AD2, nb);
                    TVR_TRY(read());
                    const double bb = hs[S_AD2];
                    const double th = r.theta, tn = rec[j + 1].theta;
                    const double num = th * (1.0 - th), den = th * th + tn;
                    theta_bar[j] += bb * ((1.0 - 2.0 * th) / den - num * 2.0 * th / (den * den));
                    theta_bar[j + 1] += bb * (-num / (den * den));
                    // theta_{j+1}: root of t^2 + (theta_j^2 - q) t - theta_j^2, q = mu_j / L_j
                    const double q = r.mu / Lj, s = 2.0 * tn + th * th - q;
                    theta_bar[j] += theta_bar[j + 1] * 2.0 * th * (1.0 - tn) / s;
                    mu_bar[j] += theta_bar[j + 1] * (tn / s) / Lj;
                    if (r.state == 0) {
                        mu_bar[j - 1] += mu_bar[j];
                    } else if (r.state == 1 && mu_bar[j] != 0.0) {
                        // mu_j = M(x^(j), y^(j)) of eq. 9
                        const double cc = mu_bar[j] / r.D, M = r.M;
                        TVR_HIP(launch_lincomb<T>(N, xj, -1.0, yj, 0.0, nullptr, DV, st));
                        TVR_TRY(project(DV, nullptr, P, nullptr, nullptr));
                        TVR_HIP(launch_backproject<T>(g, P, W, st));  // A^T A d
                        TVR_HIP(launch_lincomb<T>(N, XBC, cc, W, -cc * M, DV, XBC, st));
                        TVR_HIP(launch_tv<T>(g.nx, g.ny, g.nz, tau, cc * alpha, xj, nullptr, XBC,
                                             XBC, nullptr, G->pstride, st, nullptr));
                        TVR_HIP(launch_tv<T>(g.nx, g.ny, g.nz, tau, -cc * alpha, yj, nullptr, XBC,
                                             XBC, nullptr, G->pstride, st, nullptr));
                        TVR_HIP(launch_hessvec<T>(g.nx, g.ny, g.nz, tau, yj, DV, YBC, W, cc * M,
                                                  -cc, -cc * alpha, YBC, part, G->pstride, st,
                                                  nullptr));
                        abar += mu_bar[j] * r.B / r.D;
                    }
                } else if (j == 0 && K > 1) {
                    TVR_HIP(launch_lincomb<T>(N, XBN, 1.0, YBN, 0.0, nullptr, XBN, st));
                }
                // x^(j+1) = P_Q(y^(j) - grad f(y^(j)) / L_j)
                TVR_HIP(launch_mask<T>(N, xn, XBN, ZB, st));
                TVR_TRY(project(ZB, nullptr, P, nullptr, nullptr));
                TVR_HIP(launch_lincomb<T>(m, b_bar, 1.0 / Lj, P, 0.0, nullptr, b_bar, st));
                TVR_HIP(launch_backproject<T>(g, P, W, st));
                int nb = 0;
                TVR_HIP(launch_hessvec<T>(g.nx, g.ny, g.nz, tau, yj, ZB, YBC, W, 1.0, -1.0 / Lj,
                                          -alpha / Lj, YBC, part, G->pstride, st, &nb));
                add(S_AD1, nb);
                TVR_TRY(read());
                abar += -hs[S_AD1] / Lj;
                std::swap(XBN, XBC);
                std::swap(YBN, YBC);
                TVR_HIP(launch_lincomb<T>(N, nullptr, 0.0, nullptr, 0.0, nullptr, XBC, st));
                TVR_HIP(launch_lincomb<T>(N, nullptr, 0.0, nullptr, 0.0, nullptr, YBC, st));
            }
        }
        TVR_HIP(hipStreamSynchronize(st));
        *dl_dlogalpha = alpha * abar;
        return TVREG_OK;
    }
};

tvreg_status check_unrolled(const tvreg_geometry *G, const tvreg_solve_params *p, int32_t K,
                            int32_t ckpt)
{
    if (!G || !p)
        return fail(TVREG_EINVAL, "NULL geometry or parameters");
    if (K < 1 || ckpt < 1)
        return fail(TVREG_EINVAL, "need K >= 1 and ckpt_every >= 1");
    if (!(p->tau > 0) || !isfinite(p->tau) || !(p->alpha >= 0) || !isfinite(p->alpha))
        return fail(TVREG_EINVAL, "tau must be > 0 and alpha >= 0");
    if (!(p->L_bar > 0) || !isfinite(p->L_bar) || !(p->rho_L > 1) || p->max_trials < 1)
        return fail(TVREG_EINVAL, "need L_bar > 0, rho_L > 1, max_trials >= 1");
    // the differentiated form is UPN over the nonnegative orthant
    if (p->method != TVREG_UPN)
        return fail(TVREG_EINVAL, "the unrolled form runs UPN (method %d given)", (int)p->method);
    if (p->use_box)
        return fail(TVREG_EINVAL, "the unrolled form uses Q = {x >= 0}; use_box must be 0");
    return TVREG_OK;
}

}  // namespace

}  // namespace tvr

using namespace tvr;

extern "C" size_t tvreg_unrolled_workspace_bytes(const tvreg_geometry *G, int32_t K,
                                                 int32_t ckpt_every)
{
    if (!G || K < 1 || ckpt_every < 1)
        return 0;
    return tape_layout(G, K, ckpt_every).total;
}

extern "C" tvreg_status tvreg_upn_unrolled_fwd(const tvreg_geometry *G, const void *b,
                                               const tvreg_solve_params *p, int32_t K,
                                               int32_t ckpt_every, const double *L_replay,
                                               double *L_out, void *xK, void *tape,
                                               size_t tape_bytes, void *stream)
{
    clear_error();
    TVR_TRY(check_unrolled(G, p, K, ckpt_every));
    if (!b || !xK)
        return fail(TVREG_EINVAL, "NULL b or xK");
    if (L_replay)
        for (int j = 0; j < K; ++j)
            if (!(L_replay[j] > 0) || !isfinite(L_replay[j]))
                return fail(TVREG_EINVAL, "L_replay[%d] must be finite and > 0", j);
    const TapeLayout lay = tape_layout(G, K, ckpt_every);
    if (!tape || tape_bytes < lay.total)
        return fail(TVREG_ENOMEM, "tape of %zu bytes needed", lay.total);
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<StepRec> rec((size_t)K + 1);
    memset(rec.data(), 0, sizeof(StepRec) * rec.size());
    int stall = 0;
    auto run = [&](auto tag) -> tvreg_status {
        using T = decltype(tag);
        Unroller<T> u{};
        u.G = G;
        u.b = (const T *)b;
        u.alpha = p->alpha;
        u.tau = p->tau;
        u.K = K;
        u.ckpt = ckpt_every;
        u.st = st;
        u.ws = (char *)tape;
        u.lay = lay;
        u.N = G->N;
        u.m = G->m;
        u.part = (double *)((char *)tape + lay.part);
        u.dsum = (double *)((char *)tape + lay.sums);
        if (!u.hs.p)
            return fail(TVREG_ENOMEM, "page-locked host buffer of %d doubles", (int)S_COUNT);
        return u.forward(L_replay, L_out, (T *)xK, rec.data(), p, &stall);
    };
    const tvreg_status s = G->prec == TVREG_F64 ? run(double()) : run(float());
    if (s < 0)
        return s;
    TapeHeader h{};
    h.magic = TAPE_MAGIC;
    h.prec = (int32_t)G->prec;
    h.K = K;
    h.ckpt = ckpt_every;
    h.status = stall ? TVREG_ESTALL : TVREG_OK;
    h.N = G->N;
    h.m = G->m;
    h.alpha = p->alpha;
    h.tau = p->tau;
    TVR_HIP(hipMemcpyAsync((char *)tape + lay.header, &h, sizeof(h), hipMemcpyHostToDevice, st));
    TVR_HIP(hipMemcpyAsync((char *)tape + lay.recs, rec.data(), sizeof(StepRec) * rec.size(),
                           hipMemcpyHostToDevice, st));
    TVR_HIP(hipStreamSynchronize(st));
    return stall ? fail(TVREG_ESTALL, "BT reached max_trials") : TVREG_OK;
}

extern "C" tvreg_status tvreg_upn_unrolled_bwd(const tvreg_geometry *G, const void *b,
                                               void *tape, size_t tape_bytes, const void *xK_bar,
                                               double *dl_dlogalpha, void *dl_db, void *stream)
{
    clear_error();
    if (!G || !b || !tape || !xK_bar || !dl_dlogalpha || !dl_db)
        return fail(TVREG_EINVAL, "NULL argument");
    DeviceGuard dg(G->device);
    if (!dg.ok)
        return fail(TVREG_EDEVICE, "cannot select device %d", G->device);
    hipStream_t st = (hipStream_t)stream;
    if (tape_bytes < sizeof(TapeHeader))
        return fail(TVREG_EINVAL, "tape too small");
    TapeHeader h{};
    TVR_HIP(hipMemcpyAsync(&h, tape, sizeof(h), hipMemcpyDeviceToHost, st));
    TVR_HIP(hipStreamSynchronize(st));
    if (h.magic != TAPE_MAGIC || h.prec != (int32_t)G->prec || h.N != G->N || h.m != G->m)
        return fail(TVREG_EINVAL, "tape was not written by a forward pass on this geometry");
    if (h.status != TVREG_OK)
        return fail(TVREG_EINVAL, "the forward pass stalled; no gradient");
    const TapeLayout lay = tape_layout(G, h.K, h.ckpt);
    if (tape_bytes < lay.total)
        return fail(TVREG_EINVAL, "tape smaller than its forward pass needed");
    std::vector<StepRec> rec((size_t)h.K + 1);
    TVR_HIP(hipMemcpyAsync(rec.data(), (char *)tape + lay.recs, sizeof(StepRec) * rec.size(),
                           hipMemcpyDeviceToHost, st));
    TVR_HIP(hipStreamSynchronize(st));
    auto run = [&](auto tag) -> tvreg_status {
        using T = decltype(tag);
        Unroller<T> u{};
        u.G = G;
        u.b = (const T *)b;
        u.alpha = h.alpha;
        u.tau = h.tau;
        u.K = h.K;
        u.ckpt = h.ckpt;
        u.st = st;
        u.ws = (char *)tape;
        u.lay = lay;
        u.N = G->N;
        u.m = G->m;
        u.part = (double *)((char *)tape + lay.part);
        u.dsum = (double *)((char *)tape + lay.sums);
        if (!u.hs.p)
            return fail(TVREG_ENOMEM, "page-locked host buffer of %d doubles", (int)S_COUNT);
        return u.backward(rec.data(), (const T *)xK_bar, (T *)dl_db, dl_dlogalpha);
    };
    return G->prec == TVREG_F64 ? run(double()) : run(float());
}
