// Host side of the C ABI declared in include/ilt.h: context creation (DFT
// tables built in FP64 and rounded once to FP32, kernels copied to the
// device, all workspaces allocated up front), argument checks, and the
// stream-ordered sequences behind each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ilt_internal.h"

void set_ns_per_tick(double v);

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(ILT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int pick_kp(int P) {
    if (2 * P <= 8) return 8;
    if (2 * P <= 24) return 24;
    if (2 * P <= 40) return 40;
    return 72;
}
int round_up(int v, int m) { return (v + m - 1) / m * m; }

// BF16 round-to-nearest-even of an FP32 value, and back.
uint16_t f2bf(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
float bf2f(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
// A [Np][NZ] column table in the spectrum kernel's fragment order: for each
// 16-row group g and 16-column block nb, lane 16 q + r holds rows
// 16 g + 4 q .. + 3 of column 16 nb + r as four consecutive floats, the B
// operands of four consecutive matrix-core steps in one 16-byte load.
std::vector<float> spectrum_fragments(const float *t, int Np, int NZ) {
    std::vector<float> f((size_t)Np * NZ);
    const int NB = NZ / 16;
    for (int g = 0; g < Np / 16; ++g)
        for (int nb = 0; nb < NB; ++nb)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 4; ++e) {
                    const int x = 16 * g + 4 * (lane >> 4) + e, n = 16 * nb + (lane & 15);
                    f[(((size_t)g * NB + nb) * 64 + lane) * 4 + e] = t[(size_t)x * NZ + n];
                }
    return f;
}

// tb ([2][Np][NZ]) in the stored-field adjoint's fragment order: per
// 32-column chunk c, 16-column half xb, column block nb and part, lane
// 16 q + r holds rows 32 c + 16 xb + 4 q .. + 3 of column 16 nb + r as four
// consecutive floats.
std::vector<float> adjoint_fragments(const float *tb, int Np, int NZ) {
    std::vector<float> f((size_t)2 * Np * NZ);
    const int NB = NZ / 16;
    size_t o = 0;
    for (int c = 0; c < Np / 32; ++c)
        for (int xb = 0; xb < 2; ++xb)
            for (int nb = 0; nb < NB; ++nb)
                for (int part = 0; part < 2; ++part)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int i = 0; i < 4; ++i) {
                            const int x = 32 * c + 16 * xb + 4 * (lane >> 4) + i, n = 16 * nb + (lane & 15);
                            f[o++] = tb[((size_t)part * Np + x) * NZ + n];
                        }
    return f;
}

void split_bf(float x, uint16_t &hi, uint16_t &lo) {
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

template <typename T>
hipError_t dalloc(T **p, size_t n) {
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    e = hipMemset(v, 0, std::max<size_t>(n, 1) * sizeof(T));
    *p = static_cast<T *>(v);
    return e;
}

void free_events(ilt_ctx *c) {
    for (int i = 0; i < 2 * c->ev_cap; ++i)
        if (c->ev && c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete[] c->ev;
    delete[] c->ev_phase;
    c->ev = nullptr;
    c->ev_phase = nullptr;
    c->ev_cap = 0;
    c->n_ev = 0;
}

void free_graph(ilt_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_key_len = 0;
}

void free_ctx(ilt_ctx *c) {
    if (!c) return;
    free_events(c);
    free_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    void *ptrs[] = {c->A64, c->H64, c->w64, c->T64, c->S64, c->Y64, c->I64, c->G64, c->Q64, c->W64, c->Z64, c->g64,
                    c->phi64, c->part64,
                    c->tl, c->tb, c->tbs, c->tba, c->ta4, c->ar, c->ai, c->H, c->sw, c->coef, c->tlhl, c->tbhl, c->Yhl, c->Spart, c->S, c->Est, c->Y, c->Tg,
                    c->I, c->G, c->g, c->phi2, c->Wpart, c->W, c->edt_scratch, c->part, c->scal, c->phib,
                    c->tgtb,
                    c->tbQ, c->arQ, c->aiQ, c->Ghat, c->Ghalf, c->Ugw, c->Vpart, c->g_prev, c->dcg,
                    c->tlQ, c->Tq, c->Ipart, c->Ihat};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

int check_ctx(const ilt_ctx *c) {
    if (!c) return fail(ILT_EINVAL, "null context");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        return fail(ILT_EINVAL, "context belongs to device %d, current device is %d", c->device, dev);
    return ILT_OK;
}

int check_ptr(const void *p, const char *name, size_t align = 4) {
    if (!p) return fail(ILT_EINVAL, "%s is null", name);
    if (!aligned(p, align)) return fail(ILT_EINVAL, "%s is not %zu-byte aligned", name, align);
    return ILT_OK;
}

int check_params(const ilt_ctx *c, const ilt_params *p, bool need_loop) {
    if (!p) return fail(ILT_EINVAL, "params is null");
    if (p->n_corners < 1 || p->n_corners > 4) return fail(ILT_EINVAL, "n_corners must be 1..4");
    if (p->optimizer != 0 && p->optimizer != 1) return fail(ILT_EINVAL, "optimizer must be 0 or 1");
    for (int i = 0; i < p->n_corners; ++i) {
        const ilt_corner &k = p->corners[i];
        if (k.set < 0 || k.set >= c->n_sets) return fail(ILT_EINVAL, "corner %d uses set %d", i, k.set);
        if (!(k.dose > 0.f) || !std::isfinite(k.dose) || !(k.omega >= 0.f) || !std::isfinite(k.omega))
            return fail(ILT_EINVAL, "corner %d has a bad dose or weight", i);
    }
    if (!(p->sigma_z > 0.f) || !std::isfinite(p->i_th)) return fail(ILT_EINVAL, "bad resist parameters");
    if (need_loop) {
        if (p->iters < 0) return fail(ILT_EINVAL, "iters < 0");
        if (p->reinit_every < 0) return fail(ILT_EINVAL, "reinit_every < 0");
        if (p->iter0 < 0) return fail(ILT_EINVAL, "iter0 < 0");
    }
    if (p->dt_mode != 0 && p->dt_mode != 1) return fail(ILT_EINVAL, "dt_mode must be 0 or 1");
    if (!std::isfinite(p->eta) || p->eta < 0.f) return fail(ILT_EINVAL, "eta must be finite and >= 0");
    if (!std::isfinite(p->lambda) || !(p->eps_kappa >= 0.f)) return fail(ILT_EINVAL, "bad lambda / eps_kappa");
    if (!(p->d_lower < 0.f) || !(p->d_upper > 0.f)) return fail(ILT_EINVAL, "need d_lower < 0 < d_upper");
    return ILT_OK;
}

resist_args make_resist_args(const ilt_params *p) {
    resist_args ra{};
    ra.n_corners = p->n_corners;
    for (int i = 0; i < 4; ++i) {
        ra.cset[i] = i < p->n_corners ? p->corners[i].set : 0;
        ra.dose[i] = i < p->n_corners ? p->corners[i].dose : 1.f;
        ra.omega[i] = i < p->n_corners ? p->corners[i].omega : 0.f;
    }
    for (int s = 0; s < ILT_MAX_SETS; ++s) ra.set_used[s] = 0;
    for (int i = 0; i < p->n_corners; ++i) ra.set_used[p->corners[i].set] = 1;
    ra.sigma_z = p->sigma_z;
    ra.i_th = p->i_th;
    return ra;
}

void used_set_range(const ilt_params *p, int *lo, int *hi) {
    int a = 1 << 30, b = -1;
    for (int i = 0; i < p->n_corners; ++i) {
        a = std::min(a, p->corners[i].set);
        b = std::max(b, p->corners[i].set);
    }
    *lo = a;
    *hi = b + 1;
}

// Record the launches of one loop phase between an event pair when the
// measurement hook is on (no-op otherwise).
struct PhaseTimer {
    ilt_ctx *c;
    int slot;
    PhaseTimer(ilt_ctx *c_, int phase) : c(c_), slot(-1) {
        if (c->profiling && c->n_ev < c->ev_cap) {
            slot = c->n_ev++;
            c->ev_phase[slot] = phase;
            (void)hipEventRecord(c->ev[2 * slot], c->stream);
        }
    }
    ~PhaseTimer() {
        if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
    }
};

// partial-buffer regions (doubles)
size_t part_resist_off(const ilt_ctx *) { return 0; }
size_t part_max_off(const ilt_ctx *c) { return 4 * (size_t)resist_blocks(c); }
size_t n_image_blocks(const ilt_ctx *c) { return (size_t)(c->Np / 64) * (c->Np / 128); }
size_t part_step_off(const ilt_ctx *c) {
    return part_max_off(c) + std::max<size_t>(n_image_blocks(c), (size_t)gradmax_blocks(c));
}
// level-set step partials: {flips, non-finite count} per block
size_t part_cg_off(const ilt_ctx *c) { return part_step_off(c) + 2 * (size_t)step_blocks(c); }
size_t part_total(const ilt_ctx *c) { return part_cg_off(c) + 3 * (size_t)gradmax_blocks(c); }

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" const char *ilt_last_error(void) { return g_err.c_str(); }

extern "C" int ilt_get_dims(const ilt_ctx *c, int *N, int *P, int *K, int *n_sets) {
    if (!c) return fail(ILT_EINVAL, "null context");
    if (N) *N = c->N;
    if (P) *P = c->P;
    if (K) *K = c->K;
    if (n_sets) *n_sets = c->n_sets;
    return ILT_OK;
}

extern "C" int ilt_create(ilt_ctx **out, const ilt_optics *o, int max_batch, void *stream) {
    if (!out) return fail(ILT_EINVAL, "out is null");
    *out = nullptr;
    if (!o) return fail(ILT_EINVAL, "optics is null");
    if (max_batch < 1 || max_batch > ILT_MAX_BATCH)
        return fail(ILT_EINVAL, "max_batch=%d outside [1, %d]", max_batch, ILT_MAX_BATCH);
    if (max_batch > 1 && (o->precision != ILT_FP32 || (o->flags & ILT_FLAG_GWINDOW_ADJOINT)))
        return fail(ILT_EUNSUPPORTED, "several clips per context need ILT_FP32 without the G-window adjoint");
    const int N = o->N, P = o->P, K = o->K, ns = o->n_sets;
    if (N < 16 || N > ILT_MAX_N) return fail(ILT_EINVAL, "N=%d outside [16, %d]", N, ILT_MAX_N);
    if (P < 1 || P % 2 == 0) return fail(ILT_EINVAL, "P=%d must be odd and positive", P);
    if (P > ILT_MAX_P) return fail(ILT_EUNSUPPORTED, "P=%d above the built maximum %d", P, ILT_MAX_P);
    if (2 * P - 1 > N) return fail(ILT_EINVAL, "window 2P-1=%d exceeds N=%d", 2 * P - 1, N);
    if (K < 1 || K > ILT_MAX_K) return fail(ILT_EINVAL, "K=%d outside [1, %d]", K, ILT_MAX_K);
    if (ns < 1 || ns > ILT_MAX_SETS) return fail(ILT_EINVAL, "n_sets=%d outside [1, %d]", ns, ILT_MAX_SETS);
    if (o->precision != ILT_FP32 && o->precision != ILT_BF16X3 && o->precision != ILT_FP64)
        return fail(ILT_EUNSUPPORTED, "precision %d not built", o->precision);
    if (o->precision == ILT_FP64 && N > ILT_FP64_MAX_N)
        return fail(ILT_EUNSUPPORTED, "ILT_FP64 contexts are built for N <= %d", ILT_FP64_MAX_N);
    if (o->flags & ~(ILT_FLAG_RECOMPUTE_FIELDS | ILT_FLAG_GWINDOW_ADJOINT | ILT_FLAG_HOPKINS_FORWARD))
        return fail(ILT_EINVAL, "unknown flags 0x%x", o->flags);
    if ((o->flags & ILT_FLAG_HOPKINS_FORWARD) &&
        (!(o->flags & ILT_FLAG_GWINDOW_ADJOINT) || o->precision != ILT_FP32))
        return fail(ILT_EINVAL, "ILT_FLAG_HOPKINS_FORWARD needs ILT_FLAG_GWINDOW_ADJOINT and ILT_FP32");
    if (!o->h_kernels || !o->h_weights) return fail(ILT_EINVAL, "kernels or weights are null");
    for (int i = 0; i < ns * K; ++i)
        if (!(o->h_weights[i] >= 0.0) || !std::isfinite(o->h_weights[i]))
            return fail(ILT_EINVAL, "weight %d is negative or not finite", i);
    for (size_t i = 0; i < (size_t)ns * K * P * P * 2; ++i)
        if (!std::isfinite(o->h_kernels[i])) return fail(ILT_EINVAL, "kernel entry %zu is not finite", i);

    ilt_ctx *c = new ilt_ctx();
    std::memset(c, 0, sizeof *c);
    c->N = N; c->P = P; c->K = K; c->n_sets = ns; c->precision = o->precision;
    c->nb = max_batch;
    c->ncur = 1;
    c->Np = round_up(N, 128);
    c->KP = pick_kp(P);
    c->FB = P / 16;
    c->MIX = (P % 16) != 0 && (P % 16) <= 8;
    if ((P % 16) > 8) c->FB += 1;
    c->NZ = 32 * c->FB + 16 * c->MIX;
    c->AP = round_up(P, 16);
    c->gwin = (o->flags & ILT_FLAG_GWINDOW_ADJOINT) ? 1 : 0;
    c->hop = (o->flags & ILT_FLAG_HOPKINS_FORWARD) ? 1 : 0;
    c->Q = 2 * P - 1;
    c->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) { free_ctx(c); return fail(ILT_EDEVICE, "hipGetDevice failed"); }
    const int Np = c->Np, KP = c->KP, NZ = c->NZ, FB = c->FB, AP = c->AP;

    // DFT window matrix A[a][x] = exp(-2 pi i ((f_a x) mod N)/N), FP64 then rounded
    std::vector<float> ar((size_t)P * Np, 0.f), ai((size_t)P * Np, 0.f);
    const int cc = (P - 1) / 2;
    for (int a = 0; a < P; ++a) {
        const long long f = a - cc;
        for (int x = 0; x < N; ++x) {
            long long ph = (f * x) % N;
            if (ph < 0) ph += N;
            const double ang = -2.0 * M_PI * (double)ph / (double)N;
            ar[(size_t)a * Np + x] = (float)std::cos(ang);
            ai[(size_t)a * Np + x] = (float)std::sin(ang);
        }
    }
    std::vector<float> tl((size_t)2 * KP * Np, 0.f), tb((size_t)2 * Np * NZ, 0.f), ta4((size_t)2 * Np * AP, 0.f);
    for (int r = 0; r < P; ++r)
        for (int y = 0; y < Np; ++y) {
            const float c_ = ar[(size_t)r * Np + y], s_ = ai[(size_t)r * Np + y];
            tl[(size_t)r * Np + y] = c_;                       // L1, real rows
            tl[(size_t)(P + r) * Np + y] = s_;                 // L1, imaginary rows
            tl[(size_t)(KP + r) * Np + y] = -s_;               // L2, real rows
            tl[(size_t)(KP + P + r) * Np + y] = c_;            // L2, imaginary rows
            tb[(size_t)y * NZ + win_re(r, FB)] = c_;           // part 0: Re -> (Re, Im)
            tb[(size_t)y * NZ + win_im(r, FB)] = s_;
            tb[((size_t)Np + y) * NZ + win_re(r, FB)] = -s_;   // part 1: Im -> (Re, Im)
            tb[((size_t)Np + y) * NZ + win_im(r, FB)] = c_;
            ta4[(size_t)y * AP + r] = c_;
            ta4[((size_t)Np + y) * AP + r] = s_;
        }
    std::vector<float2> H((size_t)ns * K * P * P), coef((size_t)ns * K * P * P);
    std::vector<float> sw((size_t)ns * K);
    for (int s = 0; s < ns; ++s)
        for (int k = 0; k < K; ++k) {
            const double scale = std::sqrt(o->h_weights[s * K + k]) / ((double)N * (double)N);
            sw[(size_t)s * K + k] = (float)scale;
            for (int e = 0; e < P * P; ++e) {
                const size_t i = ((size_t)(s * K + k) * P * P + e);
                const double hr = o->h_kernels[2 * i], hi = o->h_kernels[2 * i + 1];
                H[i] = make_float2((float)hr, (float)hi);
                coef[i] = make_float2((float)(scale * hr), (float)(-scale * hi));
            }
        }

    hipError_t e = hipSuccess;
#define ALLOC(ptr, n) \
    if (e == hipSuccess) e = dalloc(&c->ptr, (n))
    ALLOC(tl, tl.size());
    ALLOC(tb, tb.size());
    ALLOC(tbs, (size_t)Np * NZ);
    ALLOC(tba, tb.size());
    ALLOC(ta4, ta4.size());
    ALLOC(ar, ar.size());
    ALLOC(ai, ai.size());
    ALLOC(H, H.size());
    ALLOC(coef, coef.size());
    ALLOC(sw, sw.size());
    const size_t nb = (size_t)max_batch;
    ALLOC(Spart, (size_t)(Np / 16) * 4 * (c->gwin ? (size_t)c->Q * c->Q * ns : (size_t)P * P) * nb);
    const bool b3 = o->precision == ILT_BF16X3;
    const bool f64 = o->precision == ILT_FP64;
    if (!b3 && !f64 && !c->gwin && !(o->flags & ILT_FLAG_RECOMPUTE_FIELDS))
        ALLOC(Est, (size_t)ns * K * (Np / 16) * (Np / 16) * 512 * nb);
    std::vector<double2> A64h, H64h;
    std::vector<double> w64h;
    if (f64) {
        A64h.resize((size_t)P * N);
        for (int a = 0; a < P; ++a) {
            const long long f = a - (P - 1) / 2;
            for (int x = 0; x < N; ++x) {
                long long ph = (f * x) % N;
                if (ph < 0) ph += N;
                const double ang = -2.0 * M_PI * (double)ph / (double)N;
                A64h[(size_t)a * N + x] = make_double2(std::cos(ang), std::sin(ang));
            }
        }
        H64h.resize((size_t)ns * K * P * P);
        for (size_t i = 0; i < H64h.size(); ++i) H64h[i] = make_double2(o->h_kernels[2 * i], o->h_kernels[2 * i + 1]);
        w64h.assign(o->h_weights, o->h_weights + (size_t)ns * K);
        ALLOC(A64, A64h.size());
        ALLOC(H64, H64h.size());
        ALLOC(w64, w64h.size());
        ALLOC(T64, (size_t)N * P);
        ALLOC(S64, (size_t)P * P);
        ALLOC(Y64, (size_t)ns * K * P * N);
        ALLOC(I64, (size_t)ns * N * N);
        ALLOC(G64, (size_t)ns * N * N);
        ALLOC(Q64, (size_t)ns * K * N * P);
        ALLOC(W64, (size_t)P * P);
        ALLOC(Z64, (size_t)P * N);
        ALLOC(g64, (size_t)N * N);
        ALLOC(phi64, (size_t)N * N);
        ALLOC(part64, (size_t)4 * 2048 + 3 * (size_t)N * ((N + 255) / 256));
    }
    std::vector<float> tbQ, arQ, aiQ;
    if (c->gwin) {
        // tables of the difference window: f_a = a - (P - 1), a in [0, Q);
        // the column table holds the columns f >= 0 only (G is real, so its
        // spectrum's other columns are conjugates), in the layout of P
        const int Q = c->Q;
        tbQ.assign((size_t)Np * NZ, 0.f);
        arQ.assign((size_t)Q * Np, 0.f);
        aiQ.assign((size_t)Q * Np, 0.f);
        for (int a = 0; a < Q; ++a) {
            const long long f = a - (P - 1);
            for (int x = 0; x < N; ++x) {
                long long ph = (f * x) % N;
                if (ph < 0) ph += N;
                const double ang = -2.0 * M_PI * (double)ph / (double)N;
                const float cr = (float)std::cos(ang), sn = (float)std::sin(ang);
                arQ[(size_t)a * Np + x] = cr;
                aiQ[(size_t)a * Np + x] = sn;
                if (f >= 0) {
                    tbQ[(size_t)x * NZ + win_re((int)f, FB)] = cr;
                    tbQ[(size_t)x * NZ + win_im((int)f, FB)] = sn;
                }
            }
        }
        ALLOC(tbQ, tbQ.size());
        ALLOC(arQ, arQ.size());
        ALLOC(aiQ, aiQ.size());
        if (c->hop) {
            ALLOC(tlQ, (size_t)KP * Np);
            ALLOC(Tq, (size_t)ns * KP * Np);
            ALLOC(Ipart, (size_t)ns * K * P * Q);
            ALLOC(Ihat, (size_t)ns * P * Q);
        }
        ALLOC(Ghat, (size_t)ns * Q * Q);
        ALLOC(Ghalf, (size_t)ns * Q * P);
        // the correlation GEMM: at most two 4-wave blocks per compute unit
        int ncu = 256;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu < 1)
            ncu = 256;
        // and at least enough ranges that one range's rows of U fit in LDS
        // beside Ghat
        const int Fpad = (P * P + 3) / 4 * 4, per_group = (gwin_ftiles(P) + 3) / 4 * ns, nchunk = Fpad / 4;
        const int cap = (GWIN_LDS_FLOATS - 2 * Q * Q) / (4 * 16 * gwin_ntiles(K));
        c->gw_groups = std::max(1, std::min(nchunk, 2 * ncu / per_group));
        c->gw_groups = std::max(c->gw_groups, (nchunk + cap - 1) / cap);
        ALLOC(Ugw, (size_t)ns * Fpad * 16 * gwin_ntiles(K));
        ALLOC(Vpart, (size_t)c->gw_groups * ns * P * P);
    }
    if (b3) {
        ALLOC(tlhl, (size_t)2 * Np * 2 * KP);
        ALLOC(tbhl, (size_t)2 * 2 * NZ * Np);
        ALLOC(Yhl, (size_t)ns * K * Np * 2 * KP);
    }
    ALLOC(S, (size_t)P * P * nb);
    ALLOC(W, (size_t)P * P * nb);
    ALLOC(Y, (size_t)ns * K * KP * Np * nb);
    ALLOC(Tg, (size_t)KP * Np * nb);
    ALLOC(I, (size_t)ns * N * N * nb);
    ALLOC(G, (size_t)ns * N * N * nb);
    ALLOC(g, (size_t)N * N * nb);
    ALLOC(g_prev, (size_t)N * N);
    ALLOC(dcg, (size_t)N * N);
    ALLOC(phi2, (size_t)N * N * nb);
    if (nb > 1) {
        ALLOC(phib, (size_t)N * N * nb);
        ALLOC(tgtb, (size_t)N * N * nb);
    }
    // W partials: one per block of the FP32 adjoint grid, or of the split-BF16 one
    c->n_wpart = std::max(ns * ((N + 31) / 32) * ((K + 3) / 4) * ILT_ST_MAX_XSPLIT, adjoint_b3_max_parts(c, ns)) * P *
                 P * 2;
    ALLOC(Wpart, (size_t)c->n_wpart * nb);
    if (e == hipSuccess) {
        unsigned char *es = nullptr;
        e = dalloc(&es, edt_scratch_bytes(N) * nb);
        c->edt_scratch = es;
    }
    c->n_part = (int)part_total(c);
    ALLOC(part, (size_t)c->n_part * nb);
    ALLOC(scal, (size_t)SC_COUNT * nb);
#undef ALLOC
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(ILT_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    if (e == hipSuccess) e = hipMemcpy(c->tl, tl.data(), tl.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->tb, tb.data(), tb.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const std::vector<float> f = spectrum_fragments(tb.data(), Np, NZ);
        e = hipMemcpy(c->tbs, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        const std::vector<float> f = adjoint_fragments(tb.data(), Np, NZ);
        e = hipMemcpy(c->tba, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(c->ta4, ta4.data(), ta4.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ar, ar.data(), ar.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ai, ai.data(), ai.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->H, H.data(), H.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->sw, sw.data(), sw.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && f64) {
        e = hipMemcpy(c->A64, A64h.data(), A64h.size() * sizeof(double2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->H64, H64h.data(), H64h.size() * sizeof(double2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->w64, w64h.data(), w64h.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && c->gwin) {
        const std::vector<float> f = spectrum_fragments(tbQ.data(), Np, NZ);
        e = hipMemcpy(c->tbQ, f.data(), f.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && c->hop) {
            // image-side table of the rows Da >= 0 of the difference window:
            // rows Re A_Q, Im A_Q at frequency Da, doubled for Da > 0 (the
            // rows Da < 0 contribute the conjugates), then zero rows
            std::vector<float> tq((size_t)KP * Np, 0.f);
            for (int d = 0; d < P; ++d) {
                const float f = d ? 2.f : 1.f;
                for (int y = 0; y < Np; ++y) {
                    tq[(size_t)d * Np + y] = f * arQ[(size_t)(P - 1 + d) * Np + y];
                    tq[(size_t)(P + d) * Np + y] = f * aiQ[(size_t)(P - 1 + d) * Np + y];
                }
            }
            e = hipMemcpy(c->tlQ, tq.data(), tq.size() * 4, hipMemcpyHostToDevice);
            // the window rows past 2P are read as zero by the image kernel
            if (e == hipSuccess) e = hipMemset(c->Tq, 0, (size_t)ns * KP * Np * 4);
        }
        if (e == hipSuccess) e = hipMemcpy(c->arQ, arQ.data(), arQ.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->aiQ, aiQ.data(), aiQ.size() * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && b3) {
        std::vector<uint16_t> lh((size_t)2 * Np * 2 * KP), bh((size_t)2 * 2 * NZ * Np);
        for (int part = 0; part < 2; ++part)
            for (int y = 0; y < Np; ++y)
                for (int r = 0; r < KP; ++r) {
                    uint16_t h, l;
                    split_bf(tl[((size_t)part * KP + r) * Np + y], h, l);
                    lh[(((size_t)part * Np + y) * 2 + 0) * KP + r] = h;
                    lh[(((size_t)part * Np + y) * 2 + 1) * KP + r] = l;
                }
        // B3 table in matrix-core fragment order, per 32-column chunk:
        // [chunk][part][n-block][hi|lo][lane][8]; lane l, element e holds
        // column n = 16 nb + l % 16, row x = 32 chunk + 4 (l / 16) + e for
        // e < 4 and 32 chunk + 16 + 4 (l / 16) + e - 4 otherwise
        const int NB = NZ / 16;
        for (int ch = 0; ch < Np / 32; ++ch)
            for (int part = 0; part < 2; ++part)
                for (int nb = 0; nb < NB; ++nb)
                    for (int l = 0; l < 64; ++l)
                        for (int el = 0; el < 8; ++el) {
                            const int n = 16 * nb + l % 16;
                            const int x = 32 * ch + (el < 4 ? 4 * (l / 16) + el : 16 + 4 * (l / 16) + el - 4);
                            uint16_t h, lo;
                            split_bf(tb[((size_t)part * Np + x) * NZ + n], h, lo);
                            const size_t base = ((((size_t)ch * 2 + part) * NB + nb) * 2) * 64 + l;
                            bh[base * 8 + el] = h;
                            bh[(base + 64) * 8 + el] = lo;
                        }
        e = hipMemcpy(c->tlhl, lh.data(), lh.size() * 2, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->tbhl, bh.data(), bh.size() * 2, hipMemcpyHostToDevice);
    }
    int rate_khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(ILT_EDEVICE, "context set-up failed: %s", hipGetErrorString(e));
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(ILT_EDEVICE, "context set-up failed: %s", hipGetErrorString(e));
    }
    c->use_graph = 1;
    c->store_fields = c->Est != nullptr;
    c->b3_xsplit = 0;
    c->st_xsplit = 0;
    c->xcd_remap = 1;
    set_ns_per_tick(rate_khz > 0 ? 1.0e6 / rate_khz : 10.0);
    *out = c;
    return ILT_OK;
}

extern "C" int ilt_destroy(ilt_ctx *c) {
    if (!c) return ILT_OK;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return ILT_OK;
}

extern "C" int litho_forward(ilt_ctx *c, const float *d_mask, int set, float *d_aerial) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_mask, "d_mask"))) return r;
    if ((r = check_ptr(d_aerial, "d_aerial"))) return r;
    if (set < 0 || set >= c->n_sets) return fail(ILT_EINVAL, "set %d outside [0, %d)", set, c->n_sets);
    HIPCHK(launch_spectrum(c, d_mask, 0));
    if (c->hop) {
        HIPCHK(launch_hopkins_spectrum(c, set, set + 1));
        HIPCHK(launch_hopkins_image(c, set, set + 1, d_aerial));
        return ILT_OK;
    }
    HIPCHK(launch_make_Y(c, set, set + 1));
    if (c->precision == ILT_BF16X3) {
        HIPCHK(launch_image_b3(c, set, set + 1, d_aerial));
    } else {
        HIPCHK(launch_image_to(c, set, set + 1, d_aerial, 0));
    }
    return ILT_OK;
}

extern "C" int litho_forward_phi(ilt_ctx *c, const float *d_phi, int set, float *d_aerial) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_phi, "d_phi"))) return r;
    if ((r = check_ptr(d_aerial, "d_aerial"))) return r;
    if (set < 0 || set >= c->n_sets) return fail(ILT_EINVAL, "set %d outside [0, %d)", set, c->n_sets);
    HIPCHK(launch_spectrum(c, d_phi, 1));
    if (c->hop) {
        HIPCHK(launch_hopkins_spectrum(c, set, set + 1));
        HIPCHK(launch_hopkins_image(c, set, set + 1, d_aerial));
        return ILT_OK;
    }
    HIPCHK(launch_make_Y(c, set, set + 1));
    if (c->precision == ILT_BF16X3) {
        HIPCHK(launch_image_b3(c, set, set + 1, d_aerial));
    } else {
        HIPCHK(launch_image_to(c, set, set + 1, d_aerial, 0));
    }
    return ILT_OK;
}

extern "C" int ilt_shifted_heaviside(const float *d_phi, float dh, long long n, float *d_out, void *stream) {
    int r;
    if ((r = check_ptr(d_phi, "d_phi"))) return r;
    if ((r = check_ptr(d_out, "d_out"))) return r;
    if (n < 0) return fail(ILT_EINVAL, "n < 0");
    if (!std::isfinite(dh)) return fail(ILT_EINVAL, "dh is not finite");
    if (n == 0) return ILT_OK;
    HIPCHK(launch_heaviside_shift(d_phi, dh, (size_t)n, d_out, static_cast<hipStream_t>(stream)));
    return ILT_OK;
}

extern "C" int litho_adjoint(ilt_ctx *c, const float *d_mask, const float *d_G, int set, float *d_out) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_mask, "d_mask"))) return r;
    if ((r = check_ptr(d_G, "d_dL_dI"))) return r;
    if ((r = check_ptr(d_out, "d_dL_dM"))) return r;
    if (set < 0 || set >= c->n_sets) return fail(ILT_EINVAL, "set %d outside [0, %d)", set, c->n_sets);
    HIPCHK(launch_spectrum(c, d_mask, 0));
    HIPCHK(launch_make_Y(c, set, set + 1));
    if (c->gwin) {
        HIPCHK(launch_adjoint_gwindow(c, d_G, 0, set, set + 1));
    } else if (c->precision == ILT_BF16X3) {
        HIPCHK(launch_adjoint_b3(c, d_G, 0, set, set + 1));
        HIPCHK(launch_window_sum(c, set, set + 1));
    } else {
        const int stored = c->Est != nullptr && c->store_fields;
        if (stored) HIPCHK(launch_image_to(c, set, set + 1, c->I + (size_t)set * c->N * c->N, 1));
        HIPCHK(launch_adjoint(c, d_G, 0, set, set + 1, stored));
        HIPCHK(launch_window_sum(c, set, set + 1));
    }
    HIPCHK(launch_gradient(c, d_out, c->part + part_max_off(c)));
    return ILT_OK;
}

extern "C" int resist_loss(ilt_ctx *c, const float *d_aerial, const unsigned char *d_target,
                           const ilt_params *p, float *d_G, double *d_stats) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_aerial, "d_aerial"))) return r;
    if ((r = check_ptr(d_target, "d_target", 1))) return r;
    if ((r = check_ptr(d_G, "d_G"))) return r;
    if (d_stats && !aligned(d_stats, 8)) return fail(ILT_EINVAL, "d_stats is not 8-byte aligned");
    if ((r = check_params(c, p, false))) return r;
    const resist_args ra = make_resist_args(p);
    const size_t npix = (size_t)c->N * c->N;
    for (int s = 0; s < c->n_sets; ++s)
        if (!ra.set_used[s]) HIPCHK(launch_fill(c, d_G + s * npix, 0.f, npix));
    HIPCHK(launch_resist(c, d_aerial, d_target, ra, d_G, c->part + part_resist_off(c)));
    HIPCHK(launch_finish_resist(c, c->part + part_resist_off(c), resist_blocks(c), c->scal, d_stats));
    return ILT_OK;
}

extern "C" int levelset_step(ilt_ctx *c, float *d_phi, const float *d_vel, const float *d_mod,
                             const ilt_params *p, double *d_stats) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_phi, "d_phi"))) return r;
    if ((r = check_ptr(d_vel, "d_vel"))) return r;
    if (d_mod && !aligned(d_mod, 4)) return fail(ILT_EINVAL, "d_mod is not 4-byte aligned");
    if (d_stats && !aligned(d_stats, 8)) return fail(ILT_EINVAL, "d_stats is not 8-byte aligned");
    if ((r = check_params(c, p, false))) return r;
    const size_t npix = (size_t)c->N * c->N;
    HIPCHK(launch_absmax(c, d_vel, c->part + part_max_off(c)));
    HIPCHK(launch_finish_dt(c, c->part + part_max_off(c), gradmax_blocks(c), p->dt_mode, p->eta, p->dt_max,
                            c->scal));
    HIPCHK(launch_levelset(c, d_phi, d_vel, d_mod, p->lambda, p->eps_kappa, c->scal, c->phi2,
                           c->part + part_step_off(c)));
    HIPCHK(launch_copy(c, d_phi, c->phi2, npix));
    HIPCHK(launch_finish_step(c, c->part + part_step_off(c), step_blocks(c), c->scal, d_stats, nullptr, 0));
    return ILT_OK;
}

extern "C" int edt_reinit(ilt_ctx *c, const float *d_phi, const unsigned char *d_mask, float *d_phi_out,
                          int *d_sqdist, const ilt_params *p) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((d_phi == nullptr) == (d_mask == nullptr))
        return fail(ILT_EINVAL, "exactly one of d_phi and d_mask must be given");
    if (d_phi && (r = check_ptr(d_phi, "d_phi"))) return r;
    if ((r = check_ptr(d_phi_out, "d_phi_out"))) return r;
    if (d_sqdist && !aligned(d_sqdist, 4)) return fail(ILT_EINVAL, "d_sqdist is not 4-byte aligned");
    if (!p) return fail(ILT_EINVAL, "params is null");
    if (!(p->d_lower < 0.f) || !(p->d_upper > 0.f)) return fail(ILT_EINVAL, "need d_lower < 0 < d_upper");
    HIPCHK(launch_edt(c, d_phi, d_mask, d_phi_out, d_sqdist, p->d_lower, p->d_upper));
    return ILT_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free TSDF: the EDT chain of edt_reinit on a scratch area that
// lives in the code object instead of a context.  The class bits and the
// per-word nearest rows for the largest side (ILT_MAX_N) take
// NOALLOC_EDT_BYTES = 6 MiB; each device the library runs on holds its own
// copy until the process ends.  Every byte the kernels read from it is
// written earlier in the same call, so nothing needs clearing, but calls that
// overlap on one device (several streams, several threads) share it and race.
namespace {
constexpr size_t NOALLOC_EDT_BYTES =
    (size_t)((ILT_MAX_N + 31) / 32) * ILT_MAX_N * (sizeof(uint32_t) + 4 * sizeof(int16_t));
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES];
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_EDT_BYTES];

namespace {
// The device address of this device's copy of `scratch`, looked up once per
// device (the host-side name is not a device address).
int noalloc_scratch(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(ILT_EUNSUPPORTED, "device %d is beyond the %d devices the scratch table holds", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ILT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return ILT_OK;
}
}  // namespace

extern "C" int edt_reinit_noalloc(int N, const float *d_phi, const unsigned char *d_mask, float d_lower,
                                  float d_upper, float *d_phi_out, int *d_sqdist, void *stream) {
    int r;
    if (N < 1 || N > ILT_MAX_N)
        return fail(ILT_EINVAL, "N=%d outside [1, %d], the largest side the %zu-byte static scratch holds", N,
                    ILT_MAX_N, NOALLOC_EDT_BYTES);
    if ((d_phi == nullptr) == (d_mask == nullptr))
        return fail(ILT_EINVAL, "exactly one of d_phi and d_mask must be given");
    if (d_phi && (r = check_ptr(d_phi, "d_phi"))) return r;
    if ((r = check_ptr(d_phi_out, "d_phi_out"))) return r;
    if (d_sqdist && !aligned(d_sqdist, 4)) return fail(ILT_EINVAL, "d_sqdist is not 4-byte aligned");
    if (!(d_lower < 0.f) || !(d_upper > 0.f)) return fail(ILT_EINVAL, "need d_lower < 0 < d_upper");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (st) {
        int cur = -1, sdev = -1;
        HIPCHK(hipGetDevice(&cur));
        HIPCHK(hipStreamGetDevice(st, &sdev));
        if (sdev != cur)
            return fail(ILT_EINVAL, "stream belongs to device %d but device %d is current", sdev, cur);
    }
    void *buf = nullptr;
    if ((r = noalloc_scratch(&buf))) return r;
    HIPCHK(launch_edt_raw(st, N, d_phi, d_mask, d_phi_out, d_sqdist, d_lower, d_upper, buf));
    return ILT_OK;
}

namespace {

// Enqueue the whole solve (init, T iterations, final metrics) on c->stream;
// d_mod: the curvature term's modulation map, or NULL for m = 1.
int enqueue_solve(ilt_ctx *c, const unsigned char *d_target, float *d_phi, const float *d_mod, const ilt_params *p,
                  double *d_trace) {
    const resist_args ra = make_resist_args(p);
    int slo, shi;
    used_set_range(p, &slo, &shi);
    const size_t npix = (size_t)c->N * c->N;
    double *pr = c->part + part_resist_off(c), *pm = c->part + part_max_off(c), *ps = c->part + part_step_off(c);
    const int stored = c->Est != nullptr && c->store_fields;
    const bool b3 = c->precision == ILT_BF16X3;
    c->n_ev = 0;
    HIPCHK(launch_set_scal(c, SC_BAD, 0.0));
    if (p->init_mode == 0) {
        PhaseTimer t(c, 7);
        HIPCHK(launch_edt(c, nullptr, d_target, d_phi, nullptr, p->d_lower, p->d_upper));
    }
    float *cur = d_phi, *nxt = c->phi2;
    for (int i = 0; i < p->iters; ++i) {
        // the loop's own iteration index: a resumed solve continues the
        // re-initialisation schedule and the trace numbering of the first
        const int gi = p->iter0 + i;
        {
            PhaseTimer t(c, 0);
            HIPCHK(launch_spectrum(c, cur, 1));
        }
        {
            PhaseTimer t(c, 1);
            if (c->hop) HIPCHK(launch_hopkins_spectrum(c, slo, shi));
            else HIPCHK(launch_make_Y(c, slo, shi));
        }
        {
            PhaseTimer t(c, 2);
            if (c->hop) HIPCHK(launch_hopkins_image(c, slo, shi, c->I + (size_t)slo * npix));
            else if (b3) HIPCHK(launch_image_b3(c, slo, shi, c->I + (size_t)slo * npix));
            else HIPCHK(launch_image_to(c, slo, shi, c->I + (size_t)slo * npix, stored));
        }
        {
            PhaseTimer t(c, 3);
            HIPCHK(launch_resist(c, c->I, d_target, ra, c->G, pr));
            HIPCHK(launch_finish_resist(c, pr, resist_blocks(c), c->scal, nullptr));
        }
        {
            PhaseTimer t(c, 4);
            if (c->gwin) HIPCHK(launch_adjoint_gwindow(c, c->G, npix, slo, shi));
            else if (b3) HIPCHK(launch_adjoint_b3(c, c->G, npix, slo, shi));
            else HIPCHK(launch_adjoint(c, c->G, npix, slo, shi, stored));
        }
        {
            PhaseTimer t(c, 5);
            if (!c->gwin) HIPCHK(launch_window_sum(c, slo, shi));
            HIPCHK(launch_gradient(c, c->g, pm));
            int nmax = (int)n_image_blocks(c);
            if (p->optimizer == 1) {
                hipError_t e = hipSuccess;
                nmax = launch_cg(c, i == 0, c->part + part_cg_off(c), pm, &e);
                HIPCHK(e);
            }
            HIPCHK(launch_finish_dt(c, pm, nmax, p->dt_mode, p->eta, p->dt_max, c->scal));
        }
        {
            PhaseTimer t(c, 6);
            HIPCHK(launch_levelset(c, cur, p->optimizer == 1 ? c->dcg : c->g, d_mod, p->lambda, p->eps_kappa,
                                   c->scal, nxt, ps));
            HIPCHK(launch_finish_step(c, ps, step_blocks(c), c->scal, nullptr,
                                      d_trace ? d_trace + (size_t)i * ILT_TRACE_W : nullptr, gi,
                                      c->ncur > 1 ? c->trace_tab : nullptr, i));
        }
        if (p->reinit_every > 0 && (gi + 1) % p->reinit_every == 0) {
            PhaseTimer t(c, 7);
            HIPCHK(launch_edt(c, nxt, nullptr, nxt, nullptr, p->d_lower, p->d_upper));
        }
        std::swap(cur, nxt);
    }
    if (cur != d_phi) HIPCHK(launch_copy(c, d_phi, cur, npix * c->ncur));
    // final metrics of [phi_T <= 0]
    HIPCHK(launch_spectrum(c, d_phi, 1));
    if (c->hop) {
        HIPCHK(launch_hopkins_spectrum(c, slo, shi));
        HIPCHK(launch_hopkins_image(c, slo, shi, c->I + (size_t)slo * npix));
    } else {
        HIPCHK(launch_make_Y(c, slo, shi));
        if (b3) {
            HIPCHK(launch_image_b3(c, slo, shi, c->I + (size_t)slo * npix));
        } else {
            HIPCHK(launch_image_to(c, slo, shi, c->I + (size_t)slo * npix, 0));
        }
    }
    HIPCHK(launch_resist(c, c->I, d_target, ra, c->G, pr));
    HIPCHK(launch_finish_resist(c, pr, resist_blocks(c), c->scal, nullptr));
    return ILT_OK;
}

static_assert(4 * sizeof(void *) + sizeof(ilt_params) <= sizeof(ilt_ctx::graph_key), "graph key buffer too small");

int graph_key(const unsigned char *d_target, const float *d_phi, const float *d_mod, const ilt_params *p,
              const double *d_trace, unsigned char *key) {
    int n = 0;
    std::memcpy(key + n, &d_target, sizeof d_target); n += sizeof d_target;
    std::memcpy(key + n, &d_phi, sizeof d_phi); n += sizeof d_phi;
    std::memcpy(key + n, &d_mod, sizeof d_mod); n += sizeof d_mod;
    std::memcpy(key + n, &d_trace, sizeof d_trace); n += sizeof d_trace;
    std::memcpy(key + n, p, sizeof *p); n += sizeof *p;
    return n;
}

int solve(ilt_ctx *c, const unsigned char *d_target, float *d_phi, const float *d_mod, const ilt_params *p,
          ilt_report *h_report, double *d_trace) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_target, "d_target", 1))) return r;
    if ((r = check_ptr(d_phi, "d_phi"))) return r;
    if (d_trace && !aligned(d_trace, 8)) return fail(ILT_EINVAL, "d_trace is not 8-byte aligned");
    if ((r = check_params(c, p, true))) return r;
    if (p->init_mode != 0 && p->init_mode != 1) return fail(ILT_EINVAL, "init_mode must be 0 or 1");

    // event pairs recorded inside a graph carry no usable timestamps, so a
    // solve with the measurement hook on launches directly
    if (c->use_graph && !c->profiling) {
        unsigned char key[sizeof c->graph_key];
        const int klen = graph_key(d_target, d_phi, d_mod, p, d_trace, key);
        if (!c->graph_exec || klen != c->graph_key_len || std::memcmp(key, c->graph_key, klen) != 0) {
            free_graph(c);
            hipStream_t user = c->stream;
            c->stream = c->cap_stream;
            hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) {
                c->stream = user;
                return fail(ILT_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
            }
            const int rc = enqueue_solve(c, d_target, d_phi, d_mod, p, d_trace);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(c->cap_stream, &g);
            c->stream = user;
            if (rc != ILT_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(ILT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            c->graph = g;
            e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                free_graph(c);
                return fail(ILT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
            std::memcpy(c->graph_key, key, klen);
            c->graph_key_len = klen;
        }
        HIPCHK(hipGraphLaunch(c->graph_exec, c->stream));
    } else {
        if ((r = enqueue_solve(c, d_target, d_phi, d_mod, p, d_trace))) return r;
    }
    double sc[SC_COUNT];
    HIPCHK(hipMemcpyAsync(sc, c->scal, sizeof sc, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (h_report) {
        h_report->iters_done = p->iters;
        h_report->loss = sc[SC_LOSS];
        h_report->l2 = (long long)sc[SC_L2];
        h_report->pvb = (long long)sc[SC_PVB];
        h_report->flips = (long long)sc[SC_FLIPS];
        h_report->status = (sc[SC_BAD] > 0.0 || !std::isfinite(sc[SC_LOSS])) ? ILT_ENUMERIC : ILT_OK;
    }
    if (sc[SC_BAD] > 0.0 || !std::isfinite(sc[SC_LOSS]))
        return fail(ILT_ENUMERIC, "non-finite loss, gradient or phi in the loop (%.0f values)", sc[SC_BAD]);
    return ILT_OK;
}

}  // namespace

// ---------------------------------------------------------------- FP64 form

namespace {

int check_f64(const ilt_ctx *c) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (c->precision != ILT_FP64) return fail(ILT_EINVAL, "the _f64 entry points need an ILT_FP64 context");
    return ILT_OK;
}

// partial-buffer regions of the FP64 form (doubles)
double *p64_resist(ilt_ctx *c) { return c->part64; }
double *p64_max(ilt_ctx *c) { return c->part64 + 4 * 2048; }
double *p64_step(ilt_ctx *c) { return c->part64 + 4 * 2048 + (size_t)c->N * rowblk64(c); }

}  // namespace

extern "C" int litho_forward_f64(ilt_ctx *c, const double *d_mask, int set, double *d_aerial) {
    int r;
    if ((r = check_f64(c))) return r;
    if ((r = check_ptr(d_mask, "d_mask", 8)) || (r = check_ptr(d_aerial, "d_aerial", 8))) return r;
    if (set < 0 || set >= c->n_sets) return fail(ILT_EINVAL, "set %d outside [0, %d)", set, c->n_sets);
    HIPCHK(launch64_spectrum(c, d_mask, 0));
    HIPCHK(launch64_image(c, set, set + 1, d_aerial));
    return ILT_OK;
}

extern "C" int litho_adjoint_f64(ilt_ctx *c, const double *d_mask, const double *d_G, int set, double *d_out) {
    int r;
    if ((r = check_f64(c))) return r;
    if ((r = check_ptr(d_mask, "d_mask", 8)) || (r = check_ptr(d_G, "d_dL_dI", 8)) ||
        (r = check_ptr(d_out, "d_dL_dM", 8)))
        return r;
    if (set < 0 || set >= c->n_sets) return fail(ILT_EINVAL, "set %d outside [0, %d)", set, c->n_sets);
    HIPCHK(launch64_spectrum(c, d_mask, 0));
    HIPCHK(launch64_make_Y(c, set, set + 1));
    HIPCHK(launch64_adjoint(c, d_G, set, set + 1));
    hipError_t e = hipSuccess;
    (void)launch64_gradient(c, d_out, p64_max(c), &e);
    HIPCHK(e);
    return ILT_OK;
}

extern "C" int ilt_solve_f64(ilt_ctx *c, const unsigned char *d_target, double *d_phi, const ilt_params *p,
                             ilt_report *h_report, double *d_trace) {
    int r;
    if ((r = check_f64(c))) return r;
    if ((r = check_ptr(d_target, "d_target", 1)) || (r = check_ptr(d_phi, "d_phi", 8))) return r;
    if (d_trace && !aligned(d_trace, 8)) return fail(ILT_EINVAL, "d_trace is not 8-byte aligned");
    if ((r = check_params(c, p, true))) return r;
    if (p->init_mode != 0 && p->init_mode != 1) return fail(ILT_EINVAL, "init_mode must be 0 or 1");
    if (p->optimizer != 0) return fail(ILT_EUNSUPPORTED, "ilt_solve_f64 runs the gradient optimizer only");
    int slo, shi;
    used_set_range(p, &slo, &shi);
    const size_t npix = (size_t)c->N * c->N;
    HIPCHK(launch_set_scal(c, SC_BAD, 0.0));
    if (p->init_mode == 0) HIPCHK(launch_edt64(c, nullptr, d_target, d_phi, nullptr, p->d_lower, p->d_upper));
    double *cur = d_phi, *nxt = c->phi64;
    hipError_t e = hipSuccess;
    for (int i = 0; i < p->iters; ++i) {
        const int gi = p->iter0 + i;
        HIPCHK(launch64_spectrum(c, cur, 1));
        HIPCHK(launch64_image(c, slo, shi, c->I64 + (size_t)slo * npix));
        HIPCHK(launch64_resist(c, c->I64, d_target, p, c->G64, p64_resist(c)));
        HIPCHK(launch_finish_resist(c, p64_resist(c), resist64_blocks(c), c->scal, nullptr));
        HIPCHK(launch64_adjoint(c, c->G64 + (size_t)slo * npix, slo, shi));
        const int nmax = launch64_gradient(c, c->g64, p64_max(c), &e);
        HIPCHK(e);
        HIPCHK(launch64_finish_dt(c, p64_max(c), nmax, p));
        const int nstep = launch64_levelset(c, cur, c->g64, p, nxt, p64_step(c), &e);
        HIPCHK(e);
        HIPCHK(launch_finish_step(c, p64_step(c), nstep, c->scal, nullptr,
                                  d_trace ? d_trace + (size_t)i * ILT_TRACE_W : nullptr, gi));
        if (p->reinit_every > 0 && (gi + 1) % p->reinit_every == 0)
            HIPCHK(launch_edt64(c, nxt, nullptr, nxt, nullptr, p->d_lower, p->d_upper));
        std::swap(cur, nxt);
    }
    if (cur != d_phi) HIPCHK(launch64_copy(c, d_phi, cur, npix));
    HIPCHK(launch64_spectrum(c, d_phi, 1));
    HIPCHK(launch64_image(c, slo, shi, c->I64 + (size_t)slo * npix));
    HIPCHK(launch64_resist(c, c->I64, d_target, p, c->G64, p64_resist(c)));
    HIPCHK(launch_finish_resist(c, p64_resist(c), resist64_blocks(c), c->scal, nullptr));
    double sc[SC_COUNT];
    HIPCHK(hipMemcpyAsync(sc, c->scal, sizeof sc, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const bool bad = sc[SC_BAD] > 0.0 || !std::isfinite(sc[SC_LOSS]);
    if (h_report) {
        h_report->iters_done = p->iters;
        h_report->loss = sc[SC_LOSS];
        h_report->l2 = (long long)sc[SC_L2];
        h_report->pvb = (long long)sc[SC_PVB];
        h_report->flips = (long long)sc[SC_FLIPS];
        h_report->status = bad ? ILT_ENUMERIC : ILT_OK;
    }
    if (bad) return fail(ILT_ENUMERIC, "non-finite loss, gradient or phi in the FP64 loop");
    return ILT_OK;
}

extern "C" int ilt_solve(ilt_ctx *c, const unsigned char *d_target, float *d_phi, const ilt_params *p,
                         ilt_report *h_report, double *d_trace) {
    return solve(c, d_target, d_phi, nullptr, p, h_report, d_trace);
}

extern "C" int ilt_solve_modulated(ilt_ctx *c, const unsigned char *d_target, float *d_phi, const float *d_mod,
                                   const ilt_params *p, ilt_report *h_report, double *d_trace) {
    int r;
    if ((r = check_ctx(c))) return r;
    if ((r = check_ptr(d_mod, "d_mod"))) return r;
    return solve(c, d_target, d_phi, d_mod, p, h_report, d_trace);
}

extern "C" int ilt_set_graph(ilt_ctx *c, int enable) {
    int r;
    if ((r = check_ctx(c))) return r;
    c->use_graph = enable ? 1 : 0;
    if (!enable) free_graph(c);
    return ILT_OK;
}

extern "C" int ilt_profile(ilt_ctx *c, int enable) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (!enable) {
        c->profiling = 0;
        return ILT_OK;
    }
    if (!c->ev) {
        const int cap = 4096;
        c->ev = new hipEvent_t[2 * cap]();
        c->ev_phase = new int[cap]();
        c->ev_cap = cap;
        for (int i = 0; i < 2 * cap; ++i)
            if (hipEventCreate(&c->ev[i]) != hipSuccess) {
                free_events(c);
                return fail(ILT_EDEVICE, "hipEventCreate failed");
            }
    }
    c->n_ev = 0;
    c->profiling = 1;
    return ILT_OK;
}

extern "C" int ilt_profile_read(ilt_ctx *c, double *h_out, int n) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (!h_out || n < 2 * ILT_N_PHASES) return fail(ILT_EINVAL, "h_out needs %d doubles", 2 * ILT_N_PHASES);
    for (int i = 0; i < 2 * ILT_N_PHASES; ++i) h_out[i] = 0.0;
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->n_ev; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        h_out[2 * c->ev_phase[i]] += ms;
        h_out[2 * c->ev_phase[i] + 1] += 1.0;
    }
    return ILT_OK;
}

// ---------------------------------------------------------------- tuning

extern "C" int ilt_get_tuning(const ilt_ctx *c, ilt_tuning *t) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (!t) return fail(ILT_EINVAL, "tuning is NULL");
    t->store_fields = c->store_fields;
    t->b3_xsplit = c->b3_xsplit;
    t->xcd_remap = c->xcd_remap;
    t->st_xsplit = c->st_xsplit;
    return ILT_OK;
}

extern "C" int ilt_set_tuning(ilt_ctx *c, const ilt_tuning *t) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (!t) return fail(ILT_EINVAL, "tuning is NULL");
    if (t->store_fields != 0 && t->store_fields != 1) return fail(ILT_EINVAL, "store_fields must be 0 or 1");
    if (t->store_fields && !c->Est)
        return fail(ILT_EINVAL, "store_fields = 1 needs the field buffer (a context without ILT_FLAG_RECOMPUTE_FIELDS, FP32)");
    if (t->b3_xsplit < 0 || t->b3_xsplit > ILT_B3_MAX_XSPLIT)
        return fail(ILT_EINVAL, "b3_xsplit must be in [0, %d]", ILT_B3_MAX_XSPLIT);
    if (t->xcd_remap != 0 && t->xcd_remap != 1) return fail(ILT_EINVAL, "xcd_remap must be 0 or 1");
    if (t->st_xsplit < 0 || t->st_xsplit > ILT_ST_MAX_XSPLIT)
        return fail(ILT_EINVAL, "st_xsplit must be in [0, %d]", ILT_ST_MAX_XSPLIT);
    c->store_fields = t->store_fields;
    c->b3_xsplit = t->b3_xsplit;
    c->xcd_remap = t->xcd_remap;
    c->st_xsplit = t->st_xsplit;
    free_graph(c);   // a captured solve used the old settings
    return ILT_OK;
}

namespace {

// Cache line prefix identifying (device architecture, problem shape, form).
std::string tune_key(const ilt_ctx *c) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[384];
    std::snprintf(buf, sizeof buf,
                  "{\"arch\": \"%s\", \"N\": %d, \"P\": %d, \"K\": %d, \"n_sets\": %d, \"precision\": %d, "
                  "\"fields_buffer\": %d, ",
                  arch.c_str(), c->N, c->P, c->K, c->n_sets, c->precision, c->Est != nullptr ? 1 : 0);
    return buf;
}

bool tune_from_cache(const char *path, const std::string &key, ilt_tuning *t, double *ms) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0) continue;
        ilt_tuning v;
        double m = 0.0;
        if (std::sscanf(line + key.size(),
                        "\"store_fields\": %d, \"b3_xsplit\": %d, \"xcd_remap\": %d, \"st_xsplit\": %d, "
                        "\"ms_per_iter\": %lf",
                        &v.store_fields, &v.b3_xsplit, &v.xcd_remap, &v.st_xsplit, &m) == 5) {
            *t = v;      // the last matching line wins
            *ms = m;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

}  // namespace

extern "C" int ilt_autotune(ilt_ctx *c, const char *cache_path, ilt_tuning *h_best, double *h_ms_per_iter) {
    int r;
    if ((r = check_ctx(c))) return r;
    const std::string key = tune_key(c);
    ilt_tuning best;
    double best_ms = 0.0;
    if (cache_path && tune_from_cache(cache_path, key, &best, &best_ms) && ilt_set_tuning(c, &best) == ILT_OK) {
        if (h_best) *h_best = best;
        if (h_ms_per_iter) *h_ms_per_iter = best_ms;
        return 1;   // taken from the cache
    }
    // candidates
    std::vector<ilt_tuning> cand;
    if (c->precision == ILT_BF16X3) {
        for (int xs : {1, 2, 4})
            for (int rm : {0, 1}) cand.push_back(ilt_tuning{0, xs, rm, 0});
    } else {
        // the column split stays at its by-size choice: on a full grid the
        // two choices differ by less than the timing noise of short solves
        if (c->Est) cand.push_back(ilt_tuning{1, 0, 1, 0});
        cand.push_back(ilt_tuning{0, 0, 1, 0});
    }
    // a synthetic clip: bars of width N/32 on a pitch of N/8 in both
    // directions inside a guard band, so every phase sees edges
    const int N = c->N;
    std::vector<unsigned char> h_t((size_t)N * N, 0);
    const int w = std::max(1, N / 32), pitch = std::max(2, N / 8), m = N / 8;
    for (int y = m; y < N - m; ++y)
        for (int x = m; x < N - m; ++x)
            h_t[(size_t)y * N + x] = ((y - m) % pitch < w) || ((x - m) % (2 * pitch) < w);
    ilt_params p{};
    p.iters = 4;
    p.reinit_every = 5;
    p.dt_mode = 0;
    p.init_mode = 0;
    p.eta = 0.85f;
    p.dt_max = 5.0f;
    p.lambda = 0.05f;
    p.sigma_z = 50.0f;
    p.i_th = 0.225f;
    p.eps_kappa = 1e-12f;
    p.d_lower = -100.0f;
    p.d_upper = 900.0f;
    p.n_corners = 1;
    p.corners[0] = ilt_corner{0, 1.0f, 1.0f};
    if (c->n_sets > 1) {
        p.n_corners = 3;
        p.corners[1] = ilt_corner{0, 1.02f, 7.5f};
        p.corners[2] = ilt_corner{1, 0.98f, 7.5f};
    }
    unsigned char *d_t = nullptr;
    float *d_phi = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&d_t, (size_t)N * N);
    if (e == hipSuccess) e = hipMalloc(&d_phi, (size_t)N * N * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(d_t, h_t.data(), h_t.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    ilt_tuning saved;
    (void)ilt_get_tuning(c, &saved);
    const int saved_prof = c->profiling;
    c->profiling = 0;
    int rc = e == hipSuccess ? ILT_OK : fail(ILT_EDEVICE, "autotune set-up: %s", hipGetErrorString(e));
    best_ms = 1e30;
    best = saved;
    // each candidate: one warm-up solve, then the fastest of three timed
    // solves (the minimum is the least disturbed by other work on the device)
    for (size_t i = 0; i < cand.size() && rc == ILT_OK; ++i) {
        if ((rc = ilt_set_tuning(c, &cand[i])) != ILT_OK) break;
        if ((rc = enqueue_solve(c, d_t, d_phi, nullptr, &p, nullptr)) != ILT_OK) break;     // warm-up
        double per_iter = 1e30;
        for (int rep = 0; rep < 3 && rc == ILT_OK && e == hipSuccess; ++rep) {
            if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
            if ((rc = enqueue_solve(c, d_t, d_phi, nullptr, &p, nullptr)) != ILT_OK) break;
            if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            per_iter = std::min(per_iter, (double)ms / p.iters);
        }
        if (rc != ILT_OK || e != hipSuccess) break;
        if (per_iter < best_ms) {
            best_ms = per_iter;
            best = cand[i];
        }
    }
    if (rc == ILT_OK && e != hipSuccess) rc = fail(ILT_EDEVICE, "autotune: %s", hipGetErrorString(e));
    c->profiling = saved_prof;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    if (d_t) (void)hipFree(d_t);
    if (d_phi) (void)hipFree(d_phi);
    if (rc != ILT_OK) {
        (void)ilt_set_tuning(c, &saved);
        return rc;
    }
    if ((rc = ilt_set_tuning(c, &best)) != ILT_OK) return rc;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (!f) return fail(ILT_EINVAL, "cannot append to the tuning cache %s", cache_path);
        std::fprintf(f,
                     "%s\"store_fields\": %d, \"b3_xsplit\": %d, \"xcd_remap\": %d, \"st_xsplit\": %d, "
                     "\"ms_per_iter\": %.6f}\n",
                     key.c_str(), best.store_fields, best.b3_xsplit, best.xcd_remap, best.st_xsplit, best_ms);
        std::fclose(f);
    }
    if (h_best) *h_best = best;
    if (h_ms_per_iter) *h_ms_per_iter = best_ms;
    return ILT_OK;
}

// ---------------------------------------------------------------- batched form
//
// Many clips, possibly of different sizes, solved in one call.  Clips of one
// size share that size's DFT tables and kernel copies through per-(size,
// lane) contexts; the clips are spread over n_lanes streams (longest clip
// first onto the least-loaded lane), so that small clips, which cannot fill
// the chip alone, run side by side.  Each lane's whole sequence of solves is
// captured into one hipGraph the first time a clip list is seen and replayed
// afterwards.  The final scalars of every clip are copied to a device report
// slot at the end of its solve and read back once.

struct ilt_batch {
    int n_sizes = 0, n_lanes = 0, max_clips = 0;
    int sizes[ILT_BATCH_MAX_SIZES] = {};
    ilt_ctx *ctx[ILT_BATCH_MAX_SIZES][ILT_BATCH_MAX_LANES] = {};
    hipStream_t user = nullptr;
    hipStream_t lane[ILT_BATCH_MAX_LANES] = {};
    hipStream_t cap[ILT_BATCH_MAX_LANES] = {};
    hipEvent_t ev_start = nullptr;
    hipEvent_t ev_lane[ILT_BATCH_MAX_LANES] = {};
    double *d_reports = nullptr;            // [max_clips][SC_COUNT]
    double *h_reports = nullptr;            // pinned mirror
    double **d_ttab = nullptr;              // [max_clips] the clips' trace pointers, in chunk order
    double **h_ttab = nullptr;              // pinned mirror
    hipGraph_t graph[ILT_BATCH_MAX_LANES] = {};
    hipGraphExec_t exec[ILT_BATCH_MAX_LANES] = {};
    std::vector<unsigned char> key;
    int use_graph = 1;
    int chunk[ILT_BATCH_MAX_SIZES] = {};    // clips per chunk of each size (<= its contexts' nb)
};

// A chunk: clips of one size with identical parameters that one context
// runs as one sequence of launches (the clip index is a grid dimension).
struct batch_chunk {
    int size = 0;                           // index into sizes
    std::vector<int> clips;                 // clip indices, in clip order
    int tab_off = 0;                        // first slot in the trace table
    double cost = 0.0;
};

namespace {

void batch_free_graphs(ilt_batch *b) {
    for (int l = 0; l < ILT_BATCH_MAX_LANES; ++l) {
        if (b->exec[l]) (void)hipGraphExecDestroy(b->exec[l]);
        if (b->graph[l]) (void)hipGraphDestroy(b->graph[l]);
        b->exec[l] = nullptr;
        b->graph[l] = nullptr;
    }
    b->key.clear();
}

void batch_free(ilt_batch *b) {
    if (!b) return;
    batch_free_graphs(b);
    for (int s = 0; s < ILT_BATCH_MAX_SIZES; ++s)
        for (int l = 0; l < ILT_BATCH_MAX_LANES; ++l)
            if (b->ctx[s][l]) {
                free_ctx(b->ctx[s][l]);
                b->ctx[s][l] = nullptr;
            }
    for (int l = 0; l < ILT_BATCH_MAX_LANES; ++l) {
        if (b->lane[l]) (void)hipStreamDestroy(b->lane[l]);
        if (b->cap[l]) (void)hipStreamDestroy(b->cap[l]);
        if (b->ev_lane[l]) (void)hipEventDestroy(b->ev_lane[l]);
    }
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    if (b->d_reports) (void)hipFree(b->d_reports);
    if (b->h_reports) (void)hipHostFree(b->h_reports);
    if (b->d_ttab) (void)hipFree(b->d_ttab);
    if (b->h_ttab) (void)hipHostFree(b->h_ttab);
    delete b;
}

int size_index(const ilt_batch *b, int N) {
    for (int s = 0; s < b->n_sizes; ++s)
        if (b->sizes[s] == N) return s;
    return -1;
}

// clips of side N per chunk: as many as make up the pixels of one 2048^2
// clip (at most 16), so that a chunk's launches fill the chip as a 2048^2
// clip's do
int chunk_capacity(int N) {
    const long long cap = (2048LL * 2048LL) / ((long long)N * N);
    return (int)std::max(1LL, std::min(16LL, cap));
}

// Chunks: clips in clip order join the last chunk of their size and
// parameters (compared byte for byte) while it has room; a conjugate-gradient
// solve runs alone.  Every chunk gets its slots of the trace table.  The
// plan is a pure function of the clip list.
void plan_chunks(const ilt_batch *b, int n, const ilt_clip *clips, std::vector<batch_chunk> &chunks) {
    chunks.clear();
    for (int i = 0; i < n; ++i) {
        const int s = size_index(b, clips[i].N);
        const int cap = clips[i].params.optimizer == 1 ? 1 : b->chunk[s];
        batch_chunk *into = nullptr;
        for (int k = (int)chunks.size() - 1; k >= 0 && !into; --k) {
            batch_chunk &ch = chunks[k];
            if (ch.size == s && (int)ch.clips.size() < cap &&
                std::memcmp(&clips[ch.clips[0]].params, &clips[i].params, sizeof(ilt_params)) == 0)
                into = &ch;
        }
        if (!into) {
            chunks.emplace_back();
            into = &chunks.back();
            into->size = s;
        }
        into->clips.push_back(i);
        into->cost += (double)clips[i].N * clips[i].N * (clips[i].params.iters + 1);
    }
    int off = 0;
    for (batch_chunk &ch : chunks) {
        ch.tab_off = off;
        off += (int)ch.clips.size();
    }
}

// Longest-processing-time-first assignment of chunks to lanes; ties keep
// the chunk order.
void plan_lanes(const ilt_batch *b, const std::vector<batch_chunk> &chunks, std::vector<int> &lane_of) {
    const int m = (int)chunks.size();
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return chunks[a].cost > chunks[c].cost; });
    std::vector<double> load(b->n_lanes, 0.0);
    lane_of.assign(m, 0);
    for (int i : order) {
        int best = 0;
        for (int l = 1; l < b->n_lanes; ++l)
            if (load[l] < load[best]) best = l;
        lane_of[i] = best;
        load[best] += chunks[i].cost;
    }
}

// Enqueue the chunks of lane l, in chunk order, on each context's current
// stream.  A chunk of one clip runs on the clip's own buffers; a larger one
// copies its clips' targets (and initial phi) into the context's clip
// buffers, runs them together and copies every phi back.
int enqueue_lane(ilt_batch *b, int l, const ilt_clip *clips, const std::vector<batch_chunk> &chunks,
                 const std::vector<int> &lane_of) {
    for (size_t k = 0; k < chunks.size(); ++k) {
        if (lane_of[k] != l) continue;
        const batch_chunk &ch = chunks[k];
        ilt_ctx *c = b->ctx[ch.size][l];
        const ilt_params &p = clips[ch.clips[0]].params;
        if (ch.clips.size() == 1) {
            const int i = ch.clips[0];
            int r = enqueue_solve(c, clips[i].d_target, clips[i].d_phi, nullptr, &p, clips[i].d_trace);
            if (r != ILT_OK) return r;
            HIPCHK(launch_copy(c, reinterpret_cast<float *>(b->d_reports + (size_t)i * SC_COUNT),
                               reinterpret_cast<const float *>(c->scal), 2 * SC_COUNT));
            continue;
        }
        const int nc = (int)ch.clips.size();
        const size_t npix = cs_npix(c);
        for (int j = 0; j < nc; ++j) {
            const ilt_clip &q = clips[ch.clips[j]];
            HIPCHK(hipMemcpyAsync(c->tgtb + j * npix, q.d_target, npix, hipMemcpyDeviceToDevice, c->stream));
            if (p.init_mode == 1)
                HIPCHK(hipMemcpyAsync(c->phib + j * npix, q.d_phi, npix * sizeof(float), hipMemcpyDeviceToDevice,
                                      c->stream));
        }
        c->ncur = nc;
        c->trace_tab = b->d_ttab + ch.tab_off;
        const int r = enqueue_solve(c, c->tgtb, c->phib, nullptr, &p, nullptr);
        c->ncur = 1;
        c->trace_tab = nullptr;
        if (r != ILT_OK) return r;
        for (int j = 0; j < nc; ++j) {
            const int i = ch.clips[j];
            HIPCHK(hipMemcpyAsync(clips[i].d_phi, c->phib + j * npix, npix * sizeof(float), hipMemcpyDeviceToDevice,
                                  c->stream));
            HIPCHK(launch_copy(c, reinterpret_cast<float *>(b->d_reports + (size_t)i * SC_COUNT),
                               reinterpret_cast<const float *>(c->scal + (size_t)j * SC_COUNT), 2 * SC_COUNT));
        }
    }
    return ILT_OK;
}

void set_lane_streams(ilt_batch *b, int l, hipStream_t s) {
    for (int z = 0; z < b->n_sizes; ++z) b->ctx[z][l]->stream = s;
}

}  // namespace

extern "C" int ilt_batch_create(ilt_batch **out, const ilt_optics *o, const int *sizes, int n_sizes,
                                int max_clips, int n_lanes, void *stream) {
    if (!out) return fail(ILT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o) return fail(ILT_EINVAL, "optics is NULL");
    if (!sizes || n_sizes < 1 || n_sizes > ILT_BATCH_MAX_SIZES)
        return fail(ILT_EINVAL, "n_sizes must be in [1, %d]", ILT_BATCH_MAX_SIZES);
    if (n_lanes < 1 || n_lanes > ILT_BATCH_MAX_LANES)
        return fail(ILT_EINVAL, "n_lanes must be in [1, %d]", ILT_BATCH_MAX_LANES);
    if (max_clips < 1 || max_clips > ILT_BATCH_MAX_CLIPS)
        return fail(ILT_EINVAL, "max_clips must be in [1, %d]", ILT_BATCH_MAX_CLIPS);
    for (int s = 0; s < n_sizes; ++s)
        for (int t = 0; t < s; ++t)
            if (sizes[s] == sizes[t]) return fail(ILT_EINVAL, "size %d listed twice", sizes[s]);
    ilt_batch *b = new (std::nothrow) ilt_batch();
    if (!b) return fail(ILT_ENOMEM, "out of host memory");
    b->n_sizes = n_sizes;
    b->n_lanes = n_lanes;
    b->max_clips = max_clips;
    b->user = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    for (int l = 0; l < n_lanes && e == hipSuccess; ++l) {
        e = hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap[l], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_lane[l], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&b->d_reports, (size_t)max_clips * SC_COUNT * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_reports, (size_t)max_clips * SC_COUNT * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->d_ttab, (size_t)max_clips * sizeof(double *));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_ttab, (size_t)max_clips * sizeof(double *));
    if (e != hipSuccess) {
        batch_free(b);
        return fail(ILT_EDEVICE, "batch set-up failed: %s", hipGetErrorString(e));
    }
    for (int s = 0; s < n_sizes; ++s) {
        b->sizes[s] = sizes[s];
        ilt_optics os = *o;
        os.N = sizes[s];
        // FP32 contexts run chunks of several clips of this size
        const bool multi = os.precision == ILT_FP32 && !(os.flags & ILT_FLAG_GWINDOW_ADJOINT);
        const int cap = multi ? std::min(chunk_capacity(sizes[s]), max_clips) : 1;
        b->chunk[s] = cap;
        for (int l = 0; l < n_lanes; ++l) {
            const int r = ilt_create(&b->ctx[s][l], &os, cap, b->lane[l]);
            if (r != ILT_OK) {
                batch_free(b);
                return r;   // message set by ilt_create
            }
        }
    }
    *out = b;
    return ILT_OK;
}

extern "C" int ilt_batch_destroy(ilt_batch *b) {
    if (!b) return fail(ILT_EINVAL, "batch is NULL");
    (void)hipDeviceSynchronize();
    batch_free(b);
    return ILT_OK;
}

extern "C" int ilt_batch_set_graph(ilt_batch *b, int enable) {
    if (!b) return fail(ILT_EINVAL, "batch is NULL");
    b->use_graph = enable ? 1 : 0;
    if (!enable) batch_free_graphs(b);
    return ILT_OK;
}

extern "C" int ilt_solve_batch(ilt_batch *b, int n, const ilt_clip *clips, ilt_report *h_reports) {
    if (!b) return fail(ILT_EINVAL, "batch is NULL");
    if (n < 1 || n > b->max_clips) return fail(ILT_EINVAL, "n must be in [1, %d]", b->max_clips);
    if (!clips) return fail(ILT_EINVAL, "clips is NULL");
    int r;
    for (int i = 0; i < n; ++i) {
        const ilt_clip &k = clips[i];
        const int s = size_index(b, k.N);
        if (s < 0) return fail(ILT_EINVAL, "clip %d: size %d was not listed at creation", i, k.N);
        if ((r = check_ptr(k.d_target, "d_target", 1))) return r;
        if ((r = check_ptr(k.d_phi, "d_phi"))) return r;
        if (k.d_trace && !aligned(k.d_trace, 8)) return fail(ILT_EINVAL, "clip %d: d_trace not 8-byte aligned", i);
        if ((r = check_params(b->ctx[s][0], &k.params, true))) return r;
        if (k.params.init_mode != 0 && k.params.init_mode != 1) return fail(ILT_EINVAL, "clip %d: bad init_mode", i);
        for (int t = 0; t < i; ++t)
            if (clips[t].d_phi == k.d_phi) return fail(ILT_EINVAL, "clips %d and %d share d_phi", t, i);
    }
    std::vector<batch_chunk> chunks;
    plan_chunks(b, n, clips, chunks);
    std::vector<int> lane_of;
    plan_lanes(b, chunks, lane_of);
    std::vector<unsigned char> key(sizeof n + (size_t)n * sizeof(ilt_clip));
    std::memcpy(key.data(), &n, sizeof n);
    std::memcpy(key.data() + sizeof n, clips, (size_t)n * sizeof(ilt_clip));

    if (!b->use_graph || key != b->key) {
        // the trace table of this clip list (read by the chunks' launches;
        // unchanged while the captured plan is replayed)
        for (const batch_chunk &ch : chunks)
            for (size_t j = 0; j < ch.clips.size(); ++j) b->h_ttab[ch.tab_off + j] = clips[ch.clips[j]].d_trace;
        HIPCHK(hipMemcpy(b->d_ttab, b->h_ttab, (size_t)n * sizeof(double *), hipMemcpyHostToDevice));
    }
    if (b->use_graph && key != b->key) {
        batch_free_graphs(b);
        for (int l = 0; l < b->n_lanes; ++l) {
            if (std::find(lane_of.begin(), lane_of.end(), l) == lane_of.end()) continue;
            set_lane_streams(b, l, b->cap[l]);
            hipError_t e = hipStreamBeginCapture(b->cap[l], hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) {
                set_lane_streams(b, l, b->lane[l]);
                batch_free_graphs(b);
                return fail(ILT_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
            }
            const int rc = enqueue_lane(b, l, clips, chunks, lane_of);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap[l], &g);
            set_lane_streams(b, l, b->lane[l]);
            b->graph[l] = g;
            if (rc != ILT_OK || e != hipSuccess) {
                batch_free_graphs(b);
                return rc != ILT_OK ? rc : fail(ILT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            }
            e = hipGraphInstantiate(&b->exec[l], g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                batch_free_graphs(b);
                return fail(ILT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
        }
        b->key = key;
    }
    HIPCHK(hipEventRecord(b->ev_start, b->user));
    for (int l = 0; l < b->n_lanes; ++l) {
        if (std::find(lane_of.begin(), lane_of.end(), l) == lane_of.end()) continue;
        HIPCHK(hipStreamWaitEvent(b->lane[l], b->ev_start, 0));
        if (b->use_graph) {
            HIPCHK(hipGraphLaunch(b->exec[l], b->lane[l]));
        } else if ((r = enqueue_lane(b, l, clips, chunks, lane_of))) {
            return r;
        }
        HIPCHK(hipEventRecord(b->ev_lane[l], b->lane[l]));
        HIPCHK(hipStreamWaitEvent(b->user, b->ev_lane[l], 0));
    }
    HIPCHK(hipMemcpyAsync(b->h_reports, b->d_reports, (size_t)n * SC_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                          b->user));
    HIPCHK(hipStreamSynchronize(b->user));
    int status = ILT_OK;
    for (int i = 0; i < n; ++i) {
        const double *sc = b->h_reports + (size_t)i * SC_COUNT;
        const bool bad = sc[SC_BAD] > 0.0 || !std::isfinite(sc[SC_LOSS]);
        if (h_reports) {
            h_reports[i].iters_done = clips[i].params.iters;
            h_reports[i].loss = sc[SC_LOSS];
            h_reports[i].l2 = (long long)sc[SC_L2];
            h_reports[i].pvb = (long long)sc[SC_PVB];
            h_reports[i].flips = (long long)sc[SC_FLIPS];
            h_reports[i].status = bad ? ILT_ENUMERIC : ILT_OK;
        }
        if (bad) status = ILT_ENUMERIC;
    }
    if (status != ILT_OK) return fail(ILT_ENUMERIC, "non-finite loss or gradient in a clip of the batch");
    return ILT_OK;
}

extern "C" int ilt_batch_autotune(ilt_batch *b, const char *cache_path, int *h_chunk, ilt_tuning *h_tuning,
                                  double *h_us_per_clip_iter) {
    if (!b) return fail(ILT_EINVAL, "batch is NULL");
    batch_free_graphs(b);   // captured with the old settings
    for (int s = 0; s < b->n_sizes; ++s) {
        ilt_ctx *c = b->ctx[s][0];
        ilt_tuning best{};
        int best_nc = 1;
        double best_us = 0.0;
        if (c->nb == 1) {
            // one clip per chunk: the single-clip tuner
            double ms = 0.0;
            const int r = ilt_autotune(c, cache_path, &best, &ms);
            if (r < 0) return r;
            best_us = 1e3 * ms;
        } else {
            // several clips per chunk: clips per chunk (the whole capacity,
            // half, a quarter) x field store and adjoint column split, timed
            // per clip and iteration on chunks of a synthetic clip
            char extra[64];
            std::snprintf(extra, sizeof extra, "\"chunk_capacity\": %d, ", c->nb);
            const std::string key = tune_key(c) + extra;
            bool cached = false;
            if (cache_path) {
                FILE *f = std::fopen(cache_path, "r");
                if (f) {
                    char line[1024];
                    while (std::fgets(line, sizeof line, f)) {
                        if (std::strncmp(line, key.c_str(), key.size()) != 0) continue;
                        ilt_tuning v;
                        int nc = 0;
                        double us = 0.0;
                        if (std::sscanf(line + key.size(),
                                        "\"chunk\": %d, \"store_fields\": %d, \"st_xsplit\": %d, "
                                        "\"us_per_clip_iter\": %lf",
                                        &nc, &v.store_fields, &v.st_xsplit, &us) == 4 &&
                            nc >= 1 && nc <= c->nb) {
                            v.b3_xsplit = 0;
                            v.xcd_remap = 1;
                            best = v;
                            best_nc = nc;
                            best_us = us;
                            cached = true;
                        }
                    }
                    std::fclose(f);
                }
            }
            if (!cached) {
                std::vector<int> ncs;
                for (int nc : {c->nb, c->nb / 2, c->nb / 4})
                    if (nc >= 1 && std::find(ncs.begin(), ncs.end(), nc) == ncs.end()) ncs.push_back(nc);
                std::vector<ilt_tuning> tun;
                if (c->Est) {
                    tun.push_back(ilt_tuning{1, 0, 1, 1});
                    tun.push_back(ilt_tuning{1, 0, 1, 2});
                }
                tun.push_back(ilt_tuning{0, 0, 1, 0});
                // the synthetic clip of ilt_autotune, in every clip slot
                const int N = c->N;
                const size_t npix = cs_npix(c);
                std::vector<unsigned char> h_t(npix, 0);
                const int w = std::max(1, N / 32), pitch = std::max(2, N / 8), m = N / 8;
                for (int y = m; y < N - m; ++y)
                    for (int x = m; x < N - m; ++x)
                        h_t[(size_t)y * N + x] = ((y - m) % pitch < w) || ((x - m) % (2 * pitch) < w);
                for (int j = 0; j < c->nb; ++j)
                    HIPCHK(hipMemcpy(c->tgtb + j * npix, h_t.data(), npix, hipMemcpyHostToDevice));
                ilt_params p{};
                p.iters = 4;
                p.reinit_every = 5;
                p.eta = 0.85f;
                p.dt_max = 5.0f;
                p.lambda = 0.05f;
                p.sigma_z = 50.0f;
                p.i_th = 0.225f;
                p.eps_kappa = 1e-12f;
                p.d_lower = -100.0f;
                p.d_upper = 900.0f;
                p.n_corners = 1;
                p.corners[0] = ilt_corner{0, 1.0f, 1.0f};
                if (c->n_sets > 1) {
                    p.n_corners = 3;
                    p.corners[1] = ilt_corner{0, 1.02f, 7.5f};
                    p.corners[2] = ilt_corner{1, 0.98f, 7.5f};
                }
                hipEvent_t e0 = nullptr, e1 = nullptr;
                HIPCHK(hipEventCreate(&e0));
                hipError_t e = hipEventCreate(&e1);
                int rc = e == hipSuccess ? ILT_OK : fail(ILT_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
                const int saved_prof = c->profiling;
                c->profiling = 0;
                best_us = 1e30;
                for (size_t ti = 0; ti < tun.size() && rc == ILT_OK; ++ti) {
                    if ((rc = ilt_set_tuning(c, &tun[ti])) != ILT_OK) break;
                    for (size_t ni = 0; ni < ncs.size() && rc == ILT_OK; ++ni) {
                        c->ncur = ncs[ni];
                        double us = 1e30;
                        // one warm-up solve, then the fastest of three
                        for (int rep = 0; rep < 4 && rc == ILT_OK && e == hipSuccess; ++rep) {
                            if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
                            if ((rc = enqueue_solve(c, c->tgtb, c->phib, nullptr, &p, nullptr)) != ILT_OK) break;
                            if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
                            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
                            float ms = 0.f;
                            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
                            if (rep > 0) us = std::min(us, 1e3 * ms / (p.iters * ncs[ni]));
                        }
                        c->ncur = 1;
                        if (rc == ILT_OK && e == hipSuccess && us < best_us) {
                            best_us = us;
                            best = tun[ti];
                            best_nc = ncs[ni];
                        }
                    }
                }
                c->ncur = 1;
                c->profiling = saved_prof;
                if (rc == ILT_OK && e != hipSuccess) rc = fail(ILT_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
                (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                if (rc != ILT_OK) return rc;
                if (cache_path) {
                    FILE *f = std::fopen(cache_path, "a");
                    if (!f) return fail(ILT_EINVAL, "cannot append to the tuning cache %s", cache_path);
                    std::fprintf(f, "%s\"chunk\": %d, \"store_fields\": %d, \"st_xsplit\": %d, "
                                    "\"us_per_clip_iter\": %.4f}\n",
                                 key.c_str(), best_nc, best.store_fields, best.st_xsplit, best_us);
                    std::fclose(f);
                }
            }
        }
        for (int l = 0; l < b->n_lanes; ++l) {
            const int r = ilt_set_tuning(b->ctx[s][l], &best);
            if (r != ILT_OK) return r;
        }
        b->chunk[s] = best_nc;
        if (h_chunk) h_chunk[s] = best_nc;
        if (h_tuning) h_tuning[s] = best;
        if (h_us_per_clip_iter) h_us_per_clip_iter[s] = best_us;
    }
    b->key.clear();
    return ILT_OK;
}

extern "C" int ilt_epe(const unsigned char *d_target, const float *d_aerial, float i_th, int N, float pitch_nm,
                       const float *h_sampling, double *d_out, void *stream) {
    int r;
    if (N < 1 || N > ILT_MAX_N) return fail(ILT_EINVAL, "N=%d outside [1, %d]", N, ILT_MAX_N);
    if ((r = check_ptr(d_target, "d_target", 1)) || (r = check_ptr(d_aerial, "d_aerial")) ||
        (r = check_ptr(d_out, "d_out", 8)))
        return r;
    if (!(pitch_nm > 0.f) || !std::isfinite(pitch_nm)) return fail(ILT_EINVAL, "pitch_nm must be positive");
    if (!std::isfinite(i_th)) return fail(ILT_EINVAL, "i_th is not finite");
    double smp[4] = {10.0, 5.0, 40.0, 15.0};
    if (h_sampling)
        for (int q = 0; q < 4; ++q) smp[q] = h_sampling[q];
    if (!(smp[0] > 0.0) || !(smp[1] >= 0.0) || !(smp[2] > 0.0) || !(smp[3] >= 0.0))
        return fail(ILT_EINVAL, "need step > 0, end >= 0, search > 0, limit >= 0");
    HIPCHK(launch_epe(d_target, d_aerial, i_th, N, (double)pitch_nm, smp[0], smp[1], smp[2], smp[3], d_out,
                      static_cast<hipStream_t>(stream)));
    return ILT_OK;
}

// ---------------------------------------------------------------- full layouts

namespace {

int check_layout(int H, int W, int N, int halo) {
    if (H < 1 || W < 1 || H > ILT_LAYOUT_MAX_SIDE || W > ILT_LAYOUT_MAX_SIDE)
        return fail(ILT_EINVAL, "layout sides must be in [1, %d]", ILT_LAYOUT_MAX_SIDE);
    if (N < 16 || N > ILT_MAX_N) return fail(ILT_EINVAL, "tile side must be in [16, %d]", ILT_MAX_N);
    if (halo < 0 || N - 2 * halo < 1) return fail(ILT_EINVAL, "need 0 <= halo and N - 2 halo >= 1");
    const long long C = N - 2 * halo;
    const long long tiles = ((H + C - 1) / C) * ((W + C - 1) / C);
    if (tiles > ILT_LAYOUT_MAX_TILES) return fail(ILT_EINVAL, "%lld tiles exceed %d", tiles, ILT_LAYOUT_MAX_TILES);
    return ILT_OK;
}

}  // namespace

extern "C" int ilt_layout_grid(int H, int W, int N, int halo, int *rows, int *cols) {
    int r;
    if ((r = check_layout(H, W, N, halo))) return r;
    if (!rows || !cols) return fail(ILT_EINVAL, "rows and cols must not be NULL");
    layout_grid_dims(H, W, N, halo, rows, cols);
    return ILT_OK;
}

extern "C" int ilt_layout_extract(const unsigned char *d_layout, int H, int W, int N, int halo,
                                  unsigned char *d_tiles, void *stream) {
    int r;
    if ((r = check_layout(H, W, N, halo))) return r;
    if ((r = check_ptr(d_layout, "d_layout", 1)) || (r = check_ptr(d_tiles, "d_tiles", 1))) return r;
    HIPCHK(launch_layout_extract(d_layout, H, W, N, halo, d_tiles, static_cast<hipStream_t>(stream)));
    return ILT_OK;
}

extern "C" int ilt_layout_stitch(const float *d_tiles, int H, int W, int N, int halo, float *d_layout,
                                 void *stream) {
    int r;
    if ((r = check_layout(H, W, N, halo))) return r;
    if ((r = check_ptr(d_tiles, "d_tiles")) || (r = check_ptr(d_layout, "d_layout"))) return r;
    HIPCHK(launch_layout_stitch(d_tiles, H, W, N, halo, d_layout, static_cast<hipStream_t>(stream)));
    return ILT_OK;
}

extern "C" int ilt_shot_count(const float *d_phi, const unsigned char *d_mask, int H, int W, long long *d_counts,
                              void *stream) {
    int r;
    if ((d_phi == nullptr) == (d_mask == nullptr))
        return fail(ILT_EINVAL, "exactly one of d_phi and d_mask must be given");
    if (d_phi && (r = check_ptr(d_phi, "d_phi"))) return r;
    if (d_mask && (r = check_ptr(d_mask, "d_mask", 1))) return r;
    if ((r = check_ptr(d_counts, "d_counts", 8))) return r;
    if (H < 1 || W < 1 || H > ILT_LAYOUT_MAX_SIDE || W > ILT_LAYOUT_MAX_SIDE)
        return fail(ILT_EINVAL, "sides must be in [1, %d]", ILT_LAYOUT_MAX_SIDE);
    HIPCHK(launch_shot_count(d_phi, d_mask, H, W, reinterpret_cast<unsigned long long *>(d_counts),
                             static_cast<hipStream_t>(stream)));
    return ILT_OK;
}

extern "C" int ilt_solve_layout(ilt_batch *b, const unsigned char *d_layout, int H, int W, int N, int halo,
                                const ilt_params *p, unsigned char *d_tile_targets, float *d_tile_phi,
                                float *d_layout_phi, ilt_report *h_reports) {
    int r;
    if (!b) return fail(ILT_EINVAL, "batch is NULL");
    if ((r = check_layout(H, W, N, halo))) return r;
    if (size_index(b, N) < 0) return fail(ILT_EINVAL, "tile side %d was not listed at batch creation", N);
    if ((r = check_ptr(d_layout, "d_layout", 1)) || (r = check_ptr(d_tile_targets, "d_tile_targets", 1)) ||
        (r = check_ptr(d_tile_phi, "d_tile_phi")) || (r = check_ptr(d_layout_phi, "d_layout_phi")))
        return r;
    if (!p) return fail(ILT_EINVAL, "params is null");
    if (p->init_mode != 0) return fail(ILT_EINVAL, "a layout solve starts every tile from TSDF(target): init_mode 0");
    int rows, cols;
    layout_grid_dims(H, W, N, halo, &rows, &cols);
    const int T = rows * cols;
    const size_t NN = (size_t)N * N;
    HIPCHK(launch_layout_extract(d_layout, H, W, N, halo, d_tile_targets, b->user));
    std::vector<ilt_clip> clips(T);
    for (int t = 0; t < T; ++t) {
        clips[t].N = N;
        clips[t].d_target = d_tile_targets + t * NN;
        clips[t].d_phi = d_tile_phi + t * NN;
        clips[t].d_trace = nullptr;
        clips[t].params = *p;
    }
    int status = ILT_OK;
    for (int off = 0; off < T; off += b->max_clips) {
        const int n = std::min(b->max_clips, T - off);
        r = ilt_solve_batch(b, n, clips.data() + off, h_reports ? h_reports + off : nullptr);
        if (r == ILT_ENUMERIC) status = r;
        else if (r != ILT_OK) return r;
    }
    HIPCHK(launch_layout_stitch(d_tile_phi, H, W, N, halo, d_layout_phi, b->user));
    HIPCHK(hipStreamSynchronize(b->user));
    if (status != ILT_OK) return fail(ILT_ENUMERIC, "non-finite loss or gradient in a tile of the layout");
    return ILT_OK;
}
