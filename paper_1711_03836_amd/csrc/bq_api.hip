// Host side of the library: the C ABI declared in include/bqhip.h.
//
// Objects: a context (device, stream, HBM budget, tuning table), gauge fields
// (links in every storage form the kernels read), operators (clover field and
// inverse for one kappa, c_SW, mu), fields (spinors in the site-tiled
// checkerboard layout) and a per-operator CG workspace.
//
// The CG state machine runs on the device: per column it keeps rho, alpha,
// beta and a status (active / stopped for a reliable update / done / failed).
// A chunk of iterations plus one reliable-update pass is a fixed sequence of
// launches, optionally captured once in a hipGraph and replayed; the host only
// reads the column states between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "bq_kernels.h"
#include "bqhip.h"

namespace bq {
// stencil instantiations, one per (storage precision, columns per thread): bq_dslash_inst.hip
hipError_t launch_hop_p0_r1(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p0_r2(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p1_r1(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p1_r2(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p1_r3(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p1_r4(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p2_r1(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p2_r2(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p2_r3(const HopLaunch& L, hipStream_t st);
hipError_t launch_hop_p2_r4(const HopLaunch& L, hipStream_t st);

hipError_t launch_hop(const HopLaunch& L, hipStream_t st)
{
    typedef hipError_t (*Fn)(const HopLaunch&, hipStream_t);
    static const Fn tab[3][4] = {{launch_hop_p0_r1, launch_hop_p0_r2, nullptr, nullptr},
                                 {launch_hop_p1_r1, launch_hop_p1_r2, launch_hop_p1_r3, launch_hop_p1_r4},
                                 {launch_hop_p2_r1, launch_hop_p2_r2, launch_hop_p2_r3, launch_hop_p2_r4}};
    // FP64 storage keeps an FP64 residual, FP32 and FP16 storage an FP32 one
    const int want_rprec = L.prec == PREC_F64 ? PREC_F64 : PREC_F32;
    if (L.prec < PREC_F64 || L.prec > PREC_F16 || L.rprec != want_rprec || L.R < 1 || L.R > 4) return hipErrorInvalidValue;
    const Fn f = tab[L.prec][L.R - 1];
    return f ? f(L, st) : hipErrorInvalidValue;
}

bool hop_variant_exists(int prec, int rprec, int recon, int R, int epi)
{
    (void)epi;
    if (R < 1) return false;
    switch (prec) {
    case PREC_F64: return rprec == PREC_F64 && (recon == 12 || recon == 18) && R <= 2;
    case PREC_F32: return rprec == PREC_F32 && (recon == 12 || recon == 18) && R <= 4;
    case PREC_F16: return rprec == PREC_F32 && recon == 12 && R <= 4;
    }
    return false;
}
}  // namespace bq

using namespace bq;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail(BQ_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define CHK(call)                         \
    do {                                  \
        int rc_ = (call);                 \
        if (rc_ != BQ_OK) return rc_;     \
    } while (0)

// ---------------------------------------------------------------------------
// context and tracked device memory
// ---------------------------------------------------------------------------

struct Tune {
    int recon, R, bs;
    int march = 0;  // > 0: t-marching stencil with segments of this many time planes, where the lattice allows
    int lds = 0;    // 1: tile-shared stencil (links and clover staged in LDS) for several column groups per tile;
                    // 2: with a lane exchange of x/y neighbours
    int order = 0;  // tile traversal of the plain and tile-shared stencils: 0 blocks of 4x4 (z,t) planes,
                    // 1 one z slab per XCD walked plane by plane in t, 2 as 1 with the column-group
                    // chunks walked one after another on each XCD
};

// The geometry a stencil launch walks for traversal order `order` (tile_at, item_of).  Order 1 cuts the
// z extent into 8 slabs of Lz / gcd(Lz, 8) planes, one per XCD (each XCD takes one contiguous
// range of logical tiles), and walks each slab t plane by t plane, so that the 8 XCDs work on
// the same few time planes at any moment and the +-t neighbours of a plane are still in the
// last-level cache when they are read again.
static Geom with_order(Geom g, int order)
{
    g.cmajor = order == 2;
    if (order < 1 || !g.blocked) return g;
    int a = g.L[2], b = 8;
    while (b) {
        const int r = a % b;
        a = b;
        b = r;
    }
    g.zb = g.L[2] / a;
    g.tb = g.L[3];
    g.nzb = g.L[2] / g.zb;
    g.inv_zb = 1.0f / (float)g.zb;
    g.inv_tb = 1.0f / (float)g.tb;
    g.inv_nzb = 1.0f / (float)g.nzb;
    return g;
}

struct bq_context_s {
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    hipStream_t stream = nullptr;
    std::map<std::pair<int, int>, Tune> tune;  // (prec, ncol) -> config
    unsigned nalloc = 0;                       // allocation counter (skews)
    bq_alloc_fn alloc = nullptr;               // caller's device allocator (NULL: hipMalloc / hipFree)
    bq_dealloc_fn dealloc = nullptr;
    void* alloc_ctx = nullptr;
    int nhandles = 0;        // live gauge fields, fields and servers created on this context
    bool closing = false;    // bq_context_destroy was called while handles were alive
};

// A context whose destroy call came while handles were alive is freed with its last handle.
static void ctx_release_handle(bq_context ctx)
{
    if (--ctx->nhandles == 0 && ctx->closing) {
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
    }
}

// Every array is laid out with its own small skew (an odd number of 128-byte lines): the
// fields, link and clover arrays have power-of-two sizes on power-of-two lattices, and
// unskewed the same tile of all of them would fall into the same L2 sets.
static const size_t kSkew = 17 * 128;

struct DevBuf {
    bq_context ctx = nullptr;
    void* raw = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (raw) {
            if (ctx->dealloc) {
                // a caller's allocator may hand the block out again at once: finish the work
                // queued on it first (hipFree synchronizes the same way)
                (void)hipDeviceSynchronize();
                ctx->dealloc(raw, ctx->alloc_ctx);
            } else {
                (void)hipFree(raw);
            }
            ctx->used -= bytes;
        }
        raw = p = nullptr;
        bytes = 0;
    }
    int alloc(bq_context c, size_t n)
    {
        release();
        ctx = c;
        if (n == 0) return BQ_OK;
        const size_t skew = (size_t)(c->nalloc++ % 31) * kSkew;
        const size_t total = n + 31 * kSkew;
        if (c->used + total > c->budget)
            return fail(BQ_ERR_OOM, "HBM budget exceeded: %zu bytes requested, %llu of %llu in use", total,
                        (unsigned long long)c->used, (unsigned long long)c->budget);
        hipError_t e = hipSuccess;
        if (c->alloc) {
            raw = c->alloc(total, c->alloc_ctx);
            if (!raw) return fail(BQ_ERR_OOM, "the caller's allocator returned NULL for %zu bytes", total);
            if (((uintptr_t)raw & 255u) != 0) {
                c->dealloc(raw, c->alloc_ctx);
                raw = nullptr;
                return fail(BQ_ERR_INVALID, "the caller's allocator returned a block not aligned to 256 bytes");
            }
        } else {
            e = hipMalloc(&raw, total);
            if (e != hipSuccess) {
                raw = nullptr;
                return fail(BQ_ERR_OOM, "hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
            }
        }
        // zero on the context stream and wait, so that work on any stream sees zeros
        e = hipMemsetAsync(raw, 0, total, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(BQ_ERR_DEVICE, "zeroing new device memory failed: %s", hipGetErrorString(e));
        p = (char*)raw + skew;
        bytes = total;
        c->used += total;
        return BQ_OK;
    }
    template <typename T> T* as() const { return (T*)p; }
};

static size_t unit_bytes(int prec) { return prec == PREC_F64 ? 16 : 8; }
// padding between the columns of a field, in storage units and in scale floats
static size_t col_pad_units(int prec) { return kSkew / (prec == PREC_F64 ? 16 : 8); }
static size_t col_pad_scales() { return kSkew / sizeof(float); }
static int spinor_nu(int prec) { return prec == PREC_F16 ? 6 : 12; }
static int clover_nu(int prec) { return prec == PREC_F16 ? 18 : 36; }
static int link_nu(int prec, int recon) { return (recon == 18 ? 9 : 6) / (prec == PREC_F16 ? 2 : 1); }

// largest distance from SU(3) (see bq_gauge_s::su3_dev) for which the two-row link form is
// kept in storage precision prec: far below that precision's rounding of the links
static double su3_tolerance(int prec) { return prec == PREC_F64 ? 1e-13 : (prec == PREC_F32 ? 1e-6 : 1e-3); }

static bool dims_ok(const int* d)
{
    if (!d) return false;
    long long v = 1;
    for (int k = 0; k < 4; k++) {
        if (d[k] < 2 || d[k] % 2) return false;
        v *= d[k];
    }
    return v / 2 < (1 << 24);  // site indices stay exact in the float-reciprocal division
}

static Geom make_geom(const int* d)
{
    Geom g{};
    for (int k = 0; k < 4; k++) g.L[k] = d[k];
    g.Lxh = d[0] / 2;
    g.Vh = g.Lxh * d[1] * d[2] * d[3];
    g.sy = g.Lxh;
    g.sz = g.Lxh * d[1];
    g.st = g.Lxh * d[1] * d[2];
    g.inv_Lxh = 1.0f / (float)g.Lxh;
    g.inv_Ly = 1.0f / (float)d[1];
    g.inv_Lz = 1.0f / (float)d[2];
    g.ntiles = pad_sites(g.Vh) / kTile;
    const int plane = g.Lxh * d[1];
    g.zb = d[2] % 4 == 0 ? 4 : (d[2] % 2 == 0 ? 2 : 1);
    g.tb = d[3] % 4 == 0 ? 4 : (d[3] % 2 == 0 ? 2 : 1);
    g.blocked = plane % kTile == 0 && (g.zb > 1 || g.tb > 1);
    g.nu = g.blocked ? plane / kTile : 1;
    g.nzb = d[2] / g.zb;
    g.inv_nu = 1.0f / (float)g.nu;
    g.inv_zb = 1.0f / (float)g.zb;
    g.inv_tb = 1.0f / (float)g.tb;
    g.inv_nzb = 1.0f / (float)g.nzb;
    return g;
}

static int sync_with(bq_context ctx, hipStream_t caller)
{
    // order ctx->stream after the caller's stream
    if (caller && caller != ctx->stream) {
        hipEvent_t ev;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, caller));
        HIPCHK(hipStreamWaitEvent(ctx->stream, ev, 0));
        HIPCHK(hipEventDestroy(ev));
    }
    return BQ_OK;
}

// ---------------------------------------------------------------------------
// gauge field, operator, field
// ---------------------------------------------------------------------------

struct LinkSet {
    DevBuf buf;
    int prec = -1, recon = 0;
    const void* U[8] = {};  // [parity*4 + mu]
};

struct bq_gauge_s {
    bq_context ctx = nullptr;
    int dims[4] = {};
    Geom g{};
    int t_bc = -1;
    int nops = 0;
    LinkSet links[5];  // F64/18, F64/12, F32/18, F32/12, F16/12 (two-row forms only where the links are SU(3))
    DevBuf B[2];       // kappa-independent clover field sum sigma (x) F per parity (built on first use)
    double su3_dev = 0;  // max over links of max(|U U^dag - 1|, |det U - 1|), measured at upload
    int nsess = 0;       // server sessions that hold this gauge field
    const LinkSet* get(int prec, int recon) const
    {
        for (const auto& l : links)
            if (l.prec == prec && l.recon == recon) return &l;
        return nullptr;
    }
};

struct Workspace;

struct bq_op_s {
    bq_gauge gauge = nullptr;
    double kappa = 0, csw = 0, mu = 0;
    DevBuf T[3][2];     // [prec][parity]
    DevBuf Tinv[3][2];  // [prec][parity]
    std::unique_ptr<Workspace> ws;
    bq_solve_stats last{};
    ~bq_op_s();
};

struct bq_field_s {
    bq_context ctx = nullptr;
    int dims[4] = {};
    Geom g{};
    int subset = BQ_FULL, prec = BQ_F64, nrhs = 1;
    int nh = 2;
    size_t half_units = 0;  // storage units per parity half per column
    size_t half_sites = 0;  // padded sites per half
    size_t cstride = 0;     // storage units between columns
    size_t sstride = 0;     // scale floats between columns (FP16)
    DevBuf data, scale;
};

// A view of nh parity halves of ncol columns of a spinor field.
struct Vec {
    void* d = nullptr;
    float* s = nullptr;
    int prec = PREC_F64;
    int nh = 1;
    size_t half_units = 0, cstride = 0, half_sites = 0, sstride = 0;
    FieldArg half(int h) const
    {
        FieldArg a;
        a.d = (char*)d + (size_t)h * half_units * unit_bytes(prec);
        a.s = s ? s + (size_t)h * half_sites : nullptr;
        a.cstride = cstride;
        a.sstride = sstride;
        return a;
    }
    FieldArg all() const { return half(0); }
    int sites() const { return (int)(nh * half_sites); }
};

static Vec field_vec(bq_field f, int first_half, int nh)
{
    Vec v;
    v.prec = f->prec;
    v.nh = nh;
    v.half_units = f->half_units;
    v.half_sites = f->half_sites;
    v.cstride = f->cstride;
    v.sstride = f->sstride;
    v.d = (char*)f->data.p + (size_t)first_half * f->half_units * unit_bytes(f->prec);
    v.s = f->prec == PREC_F16 ? f->scale.as<float>() + (size_t)first_half * f->half_sites : nullptr;
    return v;
}

// Field view of parity p of f (f must hold it)
static Vec parity_vec(bq_field f, int p) { return field_vec(f, f->subset == BQ_FULL ? p : 0, 1); }

// Strides of a work field of nh halves and ncol columns, and the bytes of its data and (FP16
// only) scale arrays.
static void vec_layout(const Geom& g, int prec, int nh, int ncol, Vec& v, size_t& data_bytes, size_t& scale_bytes)
{
    v.prec = prec;
    v.nh = nh;
    v.half_sites = pad_sites(g.Vh);
    v.half_units = v.half_sites * spinor_nu(prec);
    v.cstride = v.half_units * nh + col_pad_units(prec);
    v.sstride = v.half_sites * nh + col_pad_scales();
    v.d = nullptr;
    v.s = nullptr;
    data_bytes = v.cstride * ncol * unit_bytes(prec);
    scale_bytes = prec == PREC_F16 ? v.sstride * ncol * sizeof(float) : 0;
}

static int alloc_vec(bq_context ctx, const Geom& g, int prec, int nh, int ncol, DevBuf& data, DevBuf& scale, Vec& v)
{
    size_t db = 0, sb = 0;
    vec_layout(g, prec, nh, ncol, v, db, sb);
    CHK(data.alloc(ctx, db));
    v.d = data.p;
    if (sb) {
        CHK(scale.alloc(ctx, sb));
        v.s = scale.as<float>();
    }
    return BQ_OK;
}

// ---------------------------------------------------------------------------
// kernel configuration
// ---------------------------------------------------------------------------

static int max_R(int prec) { return prec == PREC_F64 ? 2 : 4; }

static Tune get_tune(bq_context ctx, int prec, int ncol)
{
    auto it = ctx->tune.find({prec, ncol});
    if (it != ctx->tune.end()) return it->second;
    Tune t;
    t.recon = prec == PREC_F16 ? 12 : 18;
    t.bs = ncol > 1 ? 128 : 256;
    t.R = 1;
    for (int r = std::min(max_R(prec), ncol); r >= 1; r--)
        if (ncol % r == 0) {
            t.R = r;
            break;
        }
    return t;
}

// hop launch skeleton for op, precision and tune
static HopLaunch hop_base(bq_op op, int prec, const Tune& t, int dagger, int out_parity, int ncol)
{
    HopLaunch L;
    const bq_gauge G = op->gauge;
    L.prec = prec;
    L.rprec = prec == PREC_F64 ? PREC_F64 : PREC_F32;
    // two-row links exist only for SU(3) fields (bq_gauge_upload); FP64/FP32 fall back to 18 reals
    L.recon = (t.recon == 12 && prec != PREC_F16 && !G->get(prec, 12)) ? 18 : t.recon;
    L.R = std::min(t.R, std::max(ncol, 1));
    L.bs = t.bs;
    L.march = (t.march > 0 && G->g.blocked && G->g.L[3] % t.march == 0) ? t.march : 0;
    L.lds = t.lds;
    L.dagger = dagger;
    L.g = with_order(G->g, t.order);
    L.parity = out_parity;
    L.ncol = ncol;
    const LinkSet* ls = G->get(prec, L.recon);
    for (int k = 0; k < 8; k++) L.U[k] = ls ? ls->U[k] : nullptr;
    const double ep = std::exp(op->mu), em = std::exp(-op->mu);
    L.ef = dagger ? em : ep;
    L.eb = dagger ? ep : em;
    L.tbc = G->t_bc;
    return L;
}

static int run_hop(const HopLaunch& L, hipStream_t st)
{
    for (int k = 0; k < 8; k++)
        if (!L.U[k])
            return fail(BQ_ERR_UNSUPPORTED,
                        "no %d-real link copy in precision %d: the gauge field is not SU(3) to that precision "
                        "(FP16 storage and per-column operators need the two-row form)", L.recon, L.prec);
    hipError_t e = launch_hop(L, st);
    if (e != hipSuccess)
        return fail(e == hipErrorInvalidValue ? BQ_ERR_UNSUPPORTED : BQ_ERR_DEVICE,
                    "hopping kernel (prec %d, recon %d, R %d, epi %d) launch failed: %s", L.prec, L.recon, L.R, L.epi,
                    hipGetErrorString(e));
    return BQ_OK;
}

// ---------------------------------------------------------------------------
// operator building blocks on views (precision of the views = prec)
// ---------------------------------------------------------------------------

// Per-column operators: column c of a batch uses the clover blocks and kappa of its own
// request (same gauge field and mu).  Pointers per precision and parity.
struct ColTable {
    const void* T[3][2][kMaxCols];
    const void* Tinv[3][2][kMaxCols];
    double kappa[kMaxCols];
};
// how a stencil launch scales the hop per column when a ColTable is given
enum { FK_CONST = -1, FK_KAPPA = 0, FK_MKAPPA = 1, FK_MKAPPA2 = 2 };

struct OpCall {
    bq_op op;
    int prec;
    Tune t;
    int ncol;
    const int* status = nullptr;
    int statmask = 1;
    hipStream_t st;
    const ColTable* ct = nullptr;
};

// switch a launch to per-column operators: clover per column (parity `par`, inverse or not), f by mode
static void apply_cols(const OpCall& c, HopLaunch& L, int par, bool inverse, int fk)
{
    if (!c.ct) return;
    L.percol = 1;
    if (L.recon != 12) {
        L.recon = 12;
        const LinkSet* ls = c.op->gauge->get(c.prec, 12);
        for (int k = 0; k < 8; k++) L.U[k] = ls ? ls->U[k] : nullptr;
    }
    if (c.prec == PREC_F64) L.R = 1;  // FP64 per-column variants spill above one column per thread
    for (int col = 0; col < c.ncol && col < kMaxCols; col++) {
        L.cclov[col] = inverse ? c.ct->Tinv[c.prec][par][col] : c.ct->T[c.prec][par][col];
        const double k = c.ct->kappa[col];
        L.cf[col] = fk == FK_KAPPA ? k : (fk == FK_MKAPPA ? -k : (fk == FK_MKAPPA2 ? -k * k : L.f));
    }
}

// K1: out_e = T_ee^-1 (a v_e + f D_eo in_o)   (or with D^dag)
static int k1(const OpCall& c, int dag, FieldArg in_o, FieldArg out_e, FieldArg v_e = FieldArg(), double a = 0,
              double f = 1, int fk = FK_CONST)
{
    HopLaunch L = hop_base(c.op, c.prec, c.t, dag, 0, c.ncol);
    L.epi = EPI_TINV;
    L.in = in_o;
    L.out = out_e;
    L.v = v_e;
    L.a = a;
    L.f = f;
    L.clov = c.op->Tinv[c.prec][0].p;
    L.status = c.status;
    L.statmask = c.statmask;
    apply_cols(c, L, 0, true, fk);
    return run_hop(L, c.st);
}

// out_p = C_p v_p + f D_{p,1-p} in    (+ |out|^2 partials)
static int tv(const OpCall& c, int dag, int parity, FieldArg in, FieldArg v, FieldArg out, double f, double* partial,
              int nwaves, int pstride, int fk = FK_CONST)
{
    HopLaunch L = hop_base(c.op, c.prec, c.t, dag, parity, c.ncol);
    L.epi = EPI_TV;
    L.in = in;
    L.v = v;
    L.out = out;
    L.f = f;
    L.clov = c.op->T[c.prec][parity].p;
    L.partial = partial;
    L.nwaves = nwaves;
    L.pstride = pstride;
    L.status = c.status;
    L.statmask = c.statmask;
    apply_cols(c, L, parity, false, fk);
    return run_hop(L, c.st);
}

// r_out = r_in - alpha (C_p v_p + f D_{p,1-p} in)   (+ |r_out|^2 partials)
static int tvr(const OpCall& c, int dag, int parity, FieldArg in, FieldArg v, FieldArg rin, FieldArg rout, double f,
               const double* alpha, double* partial, int nwaves, int pstride, int fk = FK_CONST)
{
    HopLaunch L = hop_base(c.op, c.prec, c.t, dag, parity, c.ncol);
    L.epi = EPI_TVR;
    L.in = in;
    L.v = v;
    L.r_in = rin;
    L.r_out = rout;
    L.f = f;
    L.alpha = alpha;
    L.clov = c.op->T[c.prec][parity].p;
    L.partial = partial;
    L.nwaves = nwaves;
    L.pstride = pstride;
    L.status = c.status;
    L.statmask = c.statmask;
    apply_cols(c, L, parity, false, fk);
    return run_hop(L, c.st);
}

// out_p = a v_p + f D_{p,1-p} in
static int hopv(const OpCall& c, int dag, int parity, FieldArg in, FieldArg out, FieldArg v, double a, double f,
                int fk = FK_CONST)
{
    HopLaunch L = hop_base(c.op, c.prec, c.t, dag, parity, c.ncol);
    L.epi = EPI_HOP;
    L.in = in;
    L.out = out;
    L.v = v;
    L.a = a;
    L.f = f;
    L.status = c.status;
    L.statmask = c.statmask;
    apply_cols(c, L, parity, false, fk);
    return run_hop(L, c.st);
}

// out_p = a v_p + f D' in with D' the hopping term whose time hops carry the factors ef (forward)
// and eb (backward) instead of e^{+-mu}; the time-boundary sign still applies
static int hop_coef(const OpCall& c, int parity, FieldArg in, FieldArg out, FieldArg v, double a, double f, double ef,
                    double eb)
{
    HopLaunch L = hop_base(c.op, c.prec, c.t, 0, parity, c.ncol);
    L.epi = EPI_HOP;
    L.in = in;
    L.out = out;
    L.v = v;
    L.a = a;
    L.f = f;
    L.ef = ef;
    L.eb = eb;
    L.status = c.status;
    L.statmask = c.statmask;
    return run_hop(L, c.st);
}

// The CG operator A = Op^dag Op: Op = Mhat on odd sites (full = 0) or M on the full lattice (full = 1).
// fwd: q = Op p with |q|^2 partials;  t is an even-parity scratch view (Mhat only).
static int op_fwd(const OpCall& c, int full, const Vec& p, const Vec& q, const Vec& t, double* partial, int hw)
{
    const double k = c.op->kappa;
    if (!full) {
        CHK(k1(c, 0, p.half(0), t.half(0)));
        return tv(c, 0, 1, t.half(0), p.half(0), q.half(0), -k * k, partial, hw, hw, c.ct ? FK_MKAPPA2 : FK_CONST);
    }
    CHK(tv(c, 0, 0, p.half(1), p.half(0), q.half(0), -k, partial, hw, 2 * hw));
    return tv(c, 0, 1, p.half(0), p.half(1), q.half(1), -k, partial ? partial + hw : nullptr, hw, 2 * hw);
}

// dag: r_out = r_in - alpha Op^dag q with |r_out|^2 partials
static int op_dag_r(const OpCall& c, int full, const Vec& q, const Vec& t, const Vec& rin, const Vec& rout,
                    const double* alpha, double* partial, int hw)
{
    const double k = c.op->kappa;
    if (!full) {
        CHK(k1(c, 1, q.half(0), t.half(0)));
        return tvr(c, 1, 1, t.half(0), q.half(0), rin.half(0), rout.half(0), -k * k, alpha, partial, hw, hw,
                   c.ct ? FK_MKAPPA2 : FK_CONST);
    }
    CHK(tvr(c, 1, 0, q.half(1), q.half(0), rin.half(0), rout.half(0), -k, alpha, partial, hw, 2 * hw));
    return tvr(c, 1, 1, q.half(0), q.half(1), rin.half(1), rout.half(1), -k, alpha, partial ? partial + hw : nullptr,
               hw, 2 * hw);
}

// ---------------------------------------------------------------------------
// CG workspace
// ---------------------------------------------------------------------------

struct Workspace {
    int ncol = 0, prec = -1, full = -1;
    // FP64 state: x, r, bp, q64 (Op x), t64 (even scratch)
    DevBuf dx, dr, dbp, dq, dt, sx, sr, sbp, sq, st_;
    Vec x, r, bp, q64, t64;
    // inner state (aliases of the FP64 vectors when prec == F64)
    DevBuf dxs, drs, dps, dqs, dts, sxs, srs, sps, sqs, sts;
    Vec xs, rs, ps, qs, ts;
    // scalars and partials
    DevBuf scal, ints, part;
    CgScalars cs{};
    double* partial = nullptr;
    double* dtmp = nullptr;  // ncol * 4 doubles for sums
    int hw = 0, pstride = 0;
    int* h_status = nullptr;  // pinned
    int* h_iters = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0;
    double graph_delta2 = -1;
    const ColTable* ct = nullptr;  // per-column operators (server sessions)
    ~Workspace()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (h_status) (void)hipHostFree(h_status);
        if (h_iters) (void)hipHostFree(h_iters);
    }
};

bq_op_s::~bq_op_s() = default;

static int ws_init(bq_context ctx, const Geom& g, int ncol, int prec, int full, Workspace* w)
{
    const int nh = full ? 2 : 1;
    w->ncol = ncol;
    w->prec = prec;
    w->full = full;
    CHK(alloc_vec(ctx, g, PREC_F64, nh, ncol, w->dx, w->sx, w->x));
    CHK(alloc_vec(ctx, g, PREC_F64, nh, ncol, w->dr, w->sr, w->r));
    CHK(alloc_vec(ctx, g, PREC_F64, nh, ncol, w->dbp, w->sbp, w->bp));
    CHK(alloc_vec(ctx, g, PREC_F64, nh, ncol, w->dq, w->sq, w->q64));
    if (!full) CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, w->dt, w->st_, w->t64));
    if (prec == PREC_F64) {
        w->xs = w->x;
        w->rs = w->r;
        w->qs = w->q64;
        w->ts = w->t64;
        CHK(alloc_vec(ctx, g, PREC_F64, nh, ncol, w->dps, w->sps, w->ps));
    } else {
        CHK(alloc_vec(ctx, g, PREC_F32, nh, ncol, w->dxs, w->sxs, w->xs));
        CHK(alloc_vec(ctx, g, PREC_F32, nh, ncol, w->drs, w->srs, w->rs));
        CHK(alloc_vec(ctx, g, prec, nh, ncol, w->dps, w->sps, w->ps));
        CHK(alloc_vec(ctx, g, prec, nh, ncol, w->dqs, w->sqs, w->qs));
        if (!full) CHK(alloc_vec(ctx, g, prec, 1, ncol, w->dts, w->sts, w->ts));
    }
    w->hw = pad_sites(g.Vh) / kTile;
    w->pstride = w->hw * nh;
    CHK(w->part.alloc(ctx, sizeof(double) * (size_t)w->pstride * ncol * 2));
    w->partial = w->part.as<double>();
    CHK(w->scal.alloc(ctx, sizeof(double) * (size_t)ncol * 10));
    CHK(w->ints.alloc(ctx, sizeof(int) * (size_t)ncol * 4));
    double* sc = w->scal.as<double>();
    int* i = w->ints.as<int>();
    w->cs.rho = sc;
    w->cs.pAp = sc + ncol;
    w->cs.alpha = sc + 2 * ncol;
    w->cs.beta = sc + 3 * ncol;
    w->cs.stop2 = sc + 4 * ncol;
    w->cs.rmax2 = sc + 5 * ncol;
    w->dtmp = sc + 6 * ncol;  // 4 * ncol
    w->cs.status = i;
    w->cs.iters = i + ncol;
    w->cs.restart = i + 2 * ncol;
    w->cs.nrel = i + 3 * ncol;
    HIPCHK(hipHostMalloc((void**)&w->h_status, sizeof(int) * ncol * 4));
    return BQ_OK;
}

static int ws_get(bq_op op, int ncol, int prec, int full, Workspace** out)
{
    Workspace* w = op->ws.get();
    if (w && w->ncol == ncol && w->prec == prec && w->full == full) {
        *out = w;
        return BQ_OK;
    }
    op->ws.reset();
    auto nw = std::make_unique<Workspace>();
    CHK(ws_init(op->gauge->ctx, op->gauge->g, ncol, prec, full, nw.get()));
    op->ws = std::move(nw);
    *out = op->ws.get();
    return BQ_OK;
}

// ---------------------------------------------------------------------------
// algorithmic byte model (every input read once, every output written once)
// ---------------------------------------------------------------------------

static double real_bytes(int prec) { return prec == PREC_F64 ? 8.0 : (prec == PREC_F32 ? 4.0 : 2.0); }
static double sp_bytes(int prec) { return 24 * real_bytes(prec) + (prec == PREC_F16 ? 4.0 : 0.0); }
static int rprec_of(int prec) { return prec == PREC_F64 ? PREC_F64 : PREC_F32; }

// links (8 per output site) + clover blocks (72 reals) read by one stencil launch over Vh output sites
static double stencil_shared(bq_op op, int prec)
{
    const Tune t = get_tune(op->gauge->ctx, prec, 1);
    return (double)op->gauge->g.Vh * (8.0 * t.recon * real_bytes(prec) + 72.0 * real_bytes(prec));
}

struct Acct {
    double bytes = 0;
    long long launches = 0;
};

// one application of A = Op^dag Op in precision prec with the residual update (per column / shared)
static double iter_col_bytes(bq_op op, int prec, int full)
{
    const double Vh = op->gauge->g.Vh, sP = sp_bytes(prec), sR = sp_bytes(rprec_of(prec));
    const double stencil = full ? 2 * Vh * 3 * sP + 2 * Vh * (2 * sP + 2 * sR)
                                : Vh * (2 * sP + 3 * sP + 2 * sP + 2 * sP + 2 * sR);
    const double update = (full ? 2 : 1) * Vh * (2 * sR + 2 * sP + sR);  // x rw, p rw, r read
    return stencil + update;
}
static double iter_shared_bytes(bq_op op, int prec) { return 4 * stencil_shared(op, prec); }
static const int kIterLaunches = 7;

// reliable pass per selected column: x += x_inner, FP64 r = b' - A x
static double rel_col_bytes(bq_op op, int prec, int full)
{
    const double Vh = op->gauge->g.Vh, n = (full ? 2 : 1) * Vh, s64 = sp_bytes(PREC_F64);
    const double accum = prec == PREC_F64 ? 0.0 : n * (2 * s64 + 2 * sp_bytes(PREC_F32));
    const double A = full ? 2 * Vh * 3 * s64 + 2 * Vh * 4 * s64 : Vh * (2 + 3 + 2 + 4) * s64;
    return accum + A;
}
// restart per restarted column: read r64, write r_inner (mixed), p rw
static double restart_col_bytes(bq_op op, int prec, int full)
{
    const double n = (full ? 2 : 1) * (double)op->gauge->g.Vh;
    return n * (sp_bytes(PREC_F64) + (prec == PREC_F64 ? 0.0 : sp_bytes(PREC_F32)) + 2 * sp_bytes(prec));
}

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------

static const int kIterMask = 1 << COL_ACTIVE;
static const int kRelMask = (1 << COL_JUST_STOPPED) | (1 << COL_STOPPED);

// one CG iteration in the inner precision
static int cg_iteration(bq_op op, Workspace* w, int prec, hipStream_t st)
{
    bq_context ctx = op->gauge->ctx;
    const int n = w->xs.sites();
    OpCall c{op, prec, get_tune(ctx, prec, w->ncol), w->ncol, w->cs.status, kIterMask, st};
    c.ct = w->ct;
    CHK(op_fwd(c, w->full, w->ps, w->qs, w->ts, w->partial, w->hw));
    HIPCHK(launch_fin_alpha(w->cs, w->partial, w->pstride, w->ncol, st));
    CHK(op_dag_r(c, w->full, w->qs, w->ts, w->rs, w->rs, w->cs.alpha, w->partial, w->hw));
    HIPCHK(launch_fin_beta(w->cs, w->partial, w->pstride, w->ncol, st));
    HIPCHK(launch_cg_update(w->xs.prec, w->xs.all(), w->ps.prec, w->ps.all(), w->rs.prec, w->rs.all(), n, w->ncol,
                            w->cs.alpha, w->cs.beta, w->cs.status, st));
    return BQ_OK;
}

// FP64 true residual r = b' - A x for the columns selected by statmask (status == nullptr: all),
// partials of |r|^2 left in w->partial
static int true_residual(bq_op op, Workspace* w, const int* status, int statmask, hipStream_t st)
{
    bq_context ctx = op->gauge->ctx;
    OpCall c{op, PREC_F64, get_tune(ctx, PREC_F64, w->ncol), w->ncol, status, statmask, st};
    c.ct = w->ct;
    CHK(op_fwd(c, w->full, w->x, w->q64, w->t64, nullptr, w->hw));
    return op_dag_r(c, w->full, w->q64, w->t64, w->bp, w->r, nullptr, w->partial, w->hw);
}

// reliable update for stopped columns: fold the inner solution into x, recompute r in FP64,
// decide done / restart on the device, restart the inner recursion from the new residual
static int reliable_pass(bq_op op, Workspace* w, int prec, hipStream_t st)
{
    const int n = w->x.sites();
    if (prec != PREC_F64) HIPCHK(launch_accum(w->xs.prec, w->xs.all(), w->x.all(), n, w->ncol, w->cs.status, kRelMask, st));
    CHK(true_residual(op, w, w->cs.status, kRelMask, st));
    HIPCHK(launch_fin_reliable(w->cs, w->partial, w->pstride, w->ncol, st));
    HIPCHK(launch_restart(w->r.all(), w->rs.prec, w->rs.all(), w->ps.prec, w->ps.all(), n, w->ncol, w->cs.beta,
                          w->cs.restart, st));
    return BQ_OK;
}

static int chunk(bq_op op, Workspace* w, int prec, int k, hipStream_t st)
{
    for (int i = 0; i < k; i++) CHK(cg_iteration(op, w, prec, st));
    return reliable_pass(op, w, prec, st);
}

// Solve A x = bp for the workspace's columns (bp already in w->bp); x left in w->x.
struct SolveAcct {
    double bytes = 0;
    long long launches = 0;
    int chunks = 0, iterations = 0;
};

static int cg_solve(bq_op op, Workspace* w, const bq_solve_params& prm, hipStream_t st, std::vector<int>& iters,
                    std::vector<int>& nrel, std::vector<int>& status, SolveAcct& acct)
{
    const int prec = w->prec;
    const int ncol = w->ncol;
    const int n = w->x.sites();
    // |b'|^2 -> rho, initial state
    HIPCHK(launch_norm2(PREC_F64, w->bp.all(), n, ncol, w->partial, w->pstride, st));
    HIPCHK(launch_fin_sum(w->partial, w->pstride, ncol, w->cs.rho, st));
    // default threshold per inner precision: an FP32 inner solve reduces its residual 100x per
    // cycle without loss (fewer FP64 reliable passes); FP16 storage limits it to about 10x
    const double delta = prm.delta > 0 ? prm.delta : (prec == PREC_F32 ? 0.01 : 0.1);
    w->cs.delta2 = prec == PREC_F64 ? 0.0 : delta * delta;
    HIPCHK(launch_cg_init(w->cs, ncol, prm.tol * prm.tol, st));
    HIPCHK(launch_zero(PREC_F64, w->x.all(), n, ncol, nullptr, 0, st));
    HIPCHK(launch_convert(PREC_F64, w->bp.all(), PREC_F64, w->r.all(), n, ncol, nullptr, 0, st));
    if (prec != PREC_F64) {
        HIPCHK(launch_zero(w->xs.prec, w->xs.all(), n, ncol, nullptr, 0, st));
        HIPCHK(launch_convert(PREC_F64, w->bp.all(), w->rs.prec, w->rs.all(), n, ncol, nullptr, 0, st));
        HIPCHK(launch_convert(w->rs.prec, w->rs.all(), w->ps.prec, w->ps.all(), n, ncol, nullptr, 0, st));
    } else {
        HIPCHK(launch_convert(PREC_F64, w->bp.all(), PREC_F64, w->ps.all(), n, ncol, nullptr, 0, st));
    }

    {
        const double s64 = sp_bytes(PREC_F64), sX = sp_bytes(rprec_of(prec)), sP = sp_bytes(prec);
        acct.bytes += (double)n * ncol * (s64 /*norm*/ + s64 /*x=0*/ + 2 * s64 /*r=b'*/);
        acct.bytes += prec == PREC_F64 ? (double)n * ncol * 2 * s64
                                       : (double)n * ncol * (sX + (s64 + sX) + (sX + sP));
        acct.launches += prec == PREC_F64 ? 6 : 8;
    }
    const int k = prm.chunk > 0 ? prm.chunk : 4;
    const bool graph = prm.use_graph != 0;
    if (graph && (w->graph == nullptr || w->graph_chunk != k || w->graph_delta2 != w->cs.delta2)) {
        if (w->graph) {
            (void)hipGraphExecDestroy(w->graph);
            w->graph = nullptr;
        }
        hipGraph_t gr;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = chunk(op, w, prec, k, st);
        hipError_t e = hipStreamEndCapture(st, &gr);
        if (rc != BQ_OK) return rc;
        if (e != hipSuccess) return fail(BQ_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&w->graph, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(BQ_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        w->graph_chunk = k;
        w->graph_delta2 = w->cs.delta2;
    }

    long done_iters = 0;
    const long maxiter = prm.maxiter > 0 ? prm.maxiter : 100000;
    // host copies of status, iters, restart, nrel (contiguous on the device)
    std::vector<int> prev(4 * ncol, 0);
    const double icol = iter_col_bytes(op, prec, w->full), ishr = iter_shared_bytes(op, prec);
    const double rcol = rel_col_bytes(op, prec, w->full), rshr = iter_shared_bytes(op, PREC_F64);
    const double scol = restart_col_bytes(op, prec, w->full);
    const int rel_launches = (prec != PREC_F64) + 4 + 2;
    while (true) {
        if (graph)
            HIPCHK(hipGraphLaunch(w->graph, st));
        else
            CHK(chunk(op, w, prec, k, st));
        done_iters += k;
        acct.launches += (long long)k * kIterLaunches + rel_launches;
        acct.chunks++;
        HIPCHK(hipMemcpyAsync(w->h_status, w->cs.status, sizeof(int) * 4 * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // Within a chunk a column is active for a prefix of the iterations (it can only stop
        // there, and restarts in the chunk's reliable pass), so the counters give exact counts.
        const int* hs = w->h_status;
        int dmax = 0, nrel_cols = 0, nrestart = 0;
        double colit = 0;
        for (int c = 0; c < ncol; c++) {
            const int di = hs[ncol + c] - prev[ncol + c];
            const int dr = hs[3 * ncol + c] - prev[3 * ncol + c];
            dmax = std::max(dmax, di);
            colit += di;
            nrel_cols += dr;
            nrestart += hs[2 * ncol + c];
        }
        acct.bytes += dmax * ishr + colit * icol;
        if (nrel_cols > 0) acct.bytes += rshr + nrel_cols * rcol + nrestart * scol;
        acct.iterations += k;
        prev.assign(hs, hs + 4 * ncol);
        bool all = true;
        for (int c = 0; c < ncol; c++)
            if (hs[c] != COL_DONE && hs[c] != COL_FAILED) all = false;
        if (all || done_iters >= maxiter) break;
    }
    // columns still running: fold the inner iterate into x
    if (prec != PREC_F64)
        HIPCHK(launch_accum(w->xs.prec, w->xs.all(), w->x.all(), n, ncol, w->cs.status,
                            (1 << COL_ACTIVE) | kRelMask, st));
    std::vector<int> h(3 * ncol);
    HIPCHK(hipMemcpyAsync(h.data(), w->cs.status, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h.data() + ncol, w->cs.iters, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h.data() + 2 * ncol, w->cs.nrel, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    status.assign(h.begin(), h.begin() + ncol);
    iters.assign(h.begin() + ncol, h.begin() + 2 * ncol);
    nrel.assign(h.begin() + 2 * ncol, h.end());
    return BQ_OK;
}

// ---------------------------------------------------------------------------
// Block CG and block multishift CG (the solver list's "block multishift cg"): one block Krylov
// space for all columns of b.  With shifts, the block residual of A + sigma_s is R xi_s for the
// residual block R of the base system (base = the smallest shift), and a run ends when every
// shift's every column has |R xi_s e_c| <= tol |b_c|.  With restarts (block CG of bq_solve) the
// FP64 residual b - A x is then recomputed and the columns that miss tol start a new run from it;
// columns found numerically dependent at the start of a run, and a run that breaks down, are
// left to the next run the same way.
// ---------------------------------------------------------------------------
static const int kBlockRuns = 8;

struct BlockOut {
    std::vector<int> iters;   // per shift and column [s * ncol + c]: iterations while it iterated
    std::vector<int> conv;    // per shift and column: recursive residual reached tol
    std::vector<int> nrel;    // per column: runs after its first
    std::vector<int> failed;  // per column: non-finite source
    int breakdowns = 0;
};

static int block_engine(bq_op op, const Vec& B, int ncol, int nshift, const double* shifts, int base, const Vec* X,
                        const bq_solve_params& prm, bool restarts, hipStream_t st, SolveAcct& acct, BlockOut& out)
{
    if (ncol < 1 || ncol > kBlockMax) return fail(BQ_ERR_UNSUPPORTED, "block CG takes 1..%d right-hand sides", kBlockMax);
    if (nshift < 1 || nshift > kMaxShifts) return fail(BQ_ERR_INVALID, "nshift must be in 1..%d", kMaxShifts);
    if (restarts && (nshift != 1 || shifts[0] != 0.0)) return fail(BQ_ERR_INVALID, "restarts need one zero shift");
    bq_context ctx = op->gauge->ctx;
    const Geom& g = op->gauge->g;
    const double kap = op->kappa;
    const int tiles = pad_sites(g.Vh) / kTile;
    const int n = (int)B.half_sites;
    const size_t units = B.half_units;
    // work fields: residual, base direction, A P, Mhat P, even scratch, a direction per other shift
    DevBuf d[5 + kMaxShifts], sc[5 + kMaxShifts];
    Vec R, P, W, Q, T;
    int nb_ = 0;
    for (Vec* v : {&R, &P, &W, &Q, &T}) {
        CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[nb_], sc[nb_], *v));
        nb_++;
    }
    BlockFields f{};
    for (int s = 0; s < nshift; s++) {
        f.x[s] = X[s].all();
        if (s == base) {
            f.p[s] = P.all();
            continue;
        }
        Vec v;
        CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[nb_], sc[nb_], v));
        nb_++;
        f.p[s] = v.all();
    }
    // device state
    const int nb = (ncol + 3) / 4;
    const int ngroups = (tiles + kGramTiles - 1) / kGramTiles;
    const size_t ns = (size_t)nshift * ncol;
    DevBuf mats, dd, ii, part, rpart;
    CHK(mats.alloc(ctx, sizeof(double2) * (size_t)kBlockMats * kBlockMax * kBlockMax));
    CHK(dd.alloc(ctx, sizeof(double) * (size_t)ncol * 2));
    CHK(ii.alloc(ctx, sizeof(int) * (BC_COUNT + ncol + 2 * ns)));
    CHK(part.alloc(ctx, sizeof(double2) * (size_t)ngroups * nb * nb * 16));
    CHK(rpart.alloc(ctx, sizeof(double) * (size_t)tiles * ncol));
    BlockState S{};
    S.mats = mats.as<double2>();
    S.thr = dd.as<double>();
    double* sums = S.thr + ncol;
    S.ctrl = ii.as<int>();
    S.colstat = S.ctrl + BC_COUNT;
    S.sstat = S.colstat + ncol;
    S.siters = S.sstat + ns;
    S.ncol = ncol;
    S.nshift = nshift;
    S.base = base;
    S.sigma_b = shifts[base];
    for (int s = 0; s < nshift; s++) S.shift[s] = shifts[s] - shifts[base];
    double2* pt = part.as<double2>();
    double* rp = rpart.as<double>();
    const double s64 = sp_bytes(PREC_F64), Vh = g.Vh;

    // thresholds (tol |b_c|)^2; zero sources are solved by x = 0, non-finite ones fail
    std::vector<double> b2(ncol), thr(ncol);
    HIPCHK(launch_norm2(PREC_F64, B.all(), n, ncol, rp, tiles, st));
    HIPCHK(launch_fin_sum(rp, tiles, ncol, sums, st));
    HIPCHK(hipMemcpyAsync(b2.data(), sums, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> cs(ncol), ss(ns, 0), si(ns, 0);
    out.iters.assign(ns, 0);
    out.conv.assign(ns, 0);
    out.nrel.assign(ncol, 0);
    out.failed.assign(ncol, 0);
    for (int c = 0; c < ncol; c++) {
        thr[c] = prm.tol * prm.tol * b2[c];
        if (!std::isfinite(b2[c])) {
            cs[c] = COL_FAILED;
            out.failed[c] = 1;
        } else if (b2[c] == 0.0) {
            cs[c] = COL_DONE;
            for (int s = 0; s < nshift; s++) ss[(size_t)s * ncol + c] = out.conv[(size_t)s * ncol + c] = 1;
        } else {
            cs[c] = COL_ACTIVE;
        }
    }
    HIPCHK(hipMemcpyAsync(S.thr, thr.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(S.sstat, ss.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(S.siters, si.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    for (int s = 0; s < nshift; s++) HIPCHK(launch_zero(PREC_F64, f.x[s], n, ncol, nullptr, 0, st));
    HIPCHK(launch_convert(PREC_F64, B.all(), PREC_F64, R.all(), n, ncol, nullptr, 0, st));
    acct.bytes += ncol * Vh * s64 * (1 + nshift + 2);
    acct.launches += 3 + nshift;

    OpCall c{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, S.colstat, 1 << COL_ACTIVE, st};
    OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, nullptr, 1, st};
    const int kchunk = prm.chunk > 0 ? prm.chunk : 8;
    const long maxiter = prm.maxiter > 0 ? prm.maxiter : 100000;
    const int per_iter = 13 + (nshift > 1);
    long total = 0;
    int runs = 0;
    std::vector<int> ctrl(BC_COUNT);
    while (true) {
        unsigned cand = 0;
        for (int c2 = 0; c2 < ncol; c2++)
            if (cs[c2] == COL_ACTIVE) cand |= 1u << c2;
        if (!cand) break;
        // a run: the candidates' Gram matrix, then the device picks the independent columns
        std::vector<int> c0(BC_COUNT, 0);
        c0[BC_MASK] = (int)cand;
        HIPCHK(hipMemcpyAsync(S.ctrl, c0.data(), sizeof(int) * BC_COUNT, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(S.colstat, cs.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, st));
        HIPCHK(launch_convert(PREC_F64, R.all(), PREC_F64, P.all(), n, ncol, nullptr, 0, st));
        for (int s = 0; s < nshift; s++)
            if (s != base) HIPCHK(launch_convert(PREC_F64, R.all(), PREC_F64, f.p[s], n, ncol, nullptr, 0, st));
        HIPCHK(launch_block_gram(R.all(), R.all(), FieldArg(), 0.0, S, g.Vh, tiles, pt, st));
        HIPCHK(launch_block_gram_fin(S, pt, tiles, BM_RR, st));
        HIPCHK(launch_block_step(S, 0, st));
        runs++;
        long run_iters = 0;
        while (true) {
            for (int it = 0; it < kchunk; it++) {
                CHK(k1(c, 0, P.all(), T.all()));
                CHK(tv(c, 0, 1, T.all(), P.all(), Q.all(), -kap * kap, nullptr, tiles, tiles));
                CHK(k1(c, 1, Q.all(), T.all()));
                CHK(tv(c, 1, 1, T.all(), Q.all(), W.all(), -kap * kap, nullptr, tiles, tiles));
                HIPCHK(launch_block_gram(P.all(), W.all(), P.all(), S.sigma_b, S, g.Vh, tiles, pt, st));
                HIPCHK(launch_block_gram_fin(S, pt, tiles, BM_PQ, st));
                HIPCHK(launch_block_step(S, 1, st));
                if (nshift > 1) HIPCHK(launch_block_shift(S, f, R.all(), units, st));
                HIPCHK(launch_block_xr(S, f.x[base], P.all(), W.all(), R.all(), units, st));
                HIPCHK(launch_block_gram(R.all(), R.all(), FieldArg(), 0.0, S, g.Vh, tiles, pt, st));
                HIPCHK(launch_block_gram_fin(S, pt, tiles, BM_RRN, st));
                HIPCHK(launch_block_step(S, 2, st));
                HIPCHK(launch_block_p(S, P.all(), R.all(), units, st));
            }
            acct.launches += (long long)kchunk * per_iter;
            acct.chunks++;
            HIPCHK(hipMemcpyAsync(ctrl.data(), S.ctrl, sizeof(int) * BC_COUNT, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            run_iters = ctrl[BC_K];
            if (ctrl[BC_STOP] || total + run_iters >= maxiter) break;
        }
        // bookkeeping of the run
        HIPCHK(hipMemcpyAsync(ss.data(), S.sstat, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(si.data(), S.siters, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const unsigned amask = (unsigned)ctrl[BC_MASK];
        const int na = ctrl[BC_NA];
        total += run_iters;
        acct.iterations += (int)run_iters;
        if (ctrl[BC_BREAK]) out.breakdowns++;
        double shift_cols = 0;
        for (int c2 = 0; c2 < ncol; c2++) {
            if (!((amask >> c2) & 1u)) continue;
            for (int s = 0; s < nshift; s++) {
                const size_t e = (size_t)s * ncol + c2;
                const int it = ss[e] ? si[e] : (int)run_iters;
                out.iters[e] += it;
                out.conv[e] = ss[e];
                if (s != base) shift_cols += it;
            }
        }
        // stencils, Gram matrices and column combinations per active column; per shift its direction
        // and solution; links and clover of the four stencil launches once per iteration
        acct.bytes += run_iters * (iter_shared_bytes(op, PREC_F64) + na * Vh * s64 * 22.0) + shift_cols * Vh * s64 * 5;
        acct.bytes += ncol * Vh * s64 * (2 + (nshift - 1) * 2 + 1);
        if (!restarts) break;
        // FP64 residual b - A x for every column
        CHK(op_fwd(c64, 0, X[base], Q, T, nullptr, tiles));
        CHK(op_dag_r(c64, 0, Q, T, B, R, nullptr, rp, tiles));
        HIPCHK(launch_fin_sum(rp, tiles, ncol, sums, st));
        std::vector<double> r2(ncol);
        HIPCHK(hipMemcpyAsync(r2.data(), sums, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        acct.bytes += iter_shared_bytes(op, PREC_F64) + ncol * Vh * s64 * 11;
        acct.launches += 5;
        bool more = false;
        for (int c2 = 0; c2 < ncol; c2++) {
            if (cs[c2] != COL_ACTIVE) continue;
            if (r2[c2] <= thr[c2]) {
                cs[c2] = COL_DONE;
                out.conv[c2] = 1;
            } else {
                out.conv[c2] = 0;
                more = true;
            }
        }
        if (!more || total >= maxiter || runs >= kBlockRuns) break;
        for (int c2 = 0; c2 < ncol; c2++)
            if (cs[c2] == COL_ACTIVE) out.nrel[c2]++;
    }
    return BQ_OK;
}

static int bcg_solve(bq_op op, Workspace* w, const bq_solve_params& prm, hipStream_t st, std::vector<int>& iters,
                     std::vector<int>& nrel, std::vector<int>& status, SolveAcct& acct)
{
    const double zero = 0.0;
    BlockOut o;
    CHK(block_engine(op, w->bp, w->ncol, 1, &zero, 0, &w->x, prm, true, st, acct, o));
    iters = o.iters;
    nrel = o.nrel;
    status.assign(w->ncol, COL_DONE);
    for (int c = 0; c < w->ncol; c++)
        if (o.failed[c]) status[c] = COL_FAILED;
    return BQ_OK;
}

// |v|^2 per column into host vector
static int norms(bq_op op, Workspace* w, const Vec& v, int ncol, std::vector<double>& out, hipStream_t st)
{
    (void)op;
    const int n = v.sites();
    const int nw = n / kTile;
    HIPCHK(launch_norm2(v.prec, v.all(), n, ncol, w->partial, nw, st));
    HIPCHK(launch_fin_sum(w->partial, nw, ncol, w->dtmp, st));
    out.resize(ncol);
    HIPCHK(hipMemcpyAsync(out.data(), w->dtmp, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return BQ_OK;
}

// Solve on views: b (FULL for SYS_M / FULL_NORMAL, ODD for NORMAL), x likewise (FP64).
static int solve_views(bq_op op, const Vec& b_even, const Vec& b_odd, const Vec& x_even, const Vec& x_odd, int ncol,
                       const bq_solve_params& prm, bq_solve_info* info, hipStream_t st, SolveAcct& acct)
{
    const int sys = prm.system;
    const int full = sys == BQ_SYS_FULL_NORMAL;
    Workspace* w;
    CHK(ws_get(op, ncol, prm.inner_prec, full, &w));
    bq_context ctx = op->gauge->ctx;
    OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, nullptr, 1, st};
    const double kap = op->kappa;
    const int hw = w->hw;

    // b' of the CG system
    {
        const double Vh = op->gauge->g.Vh, s64 = sp_bytes(PREC_F64), sh = stencil_shared(op, PREC_F64);
        const double C64 = Vh * 72 * 8.0;
        if (sys == BQ_SYS_M) {
            acct.bytes += C64 + ncol * Vh * 2 * s64;              // T_ee^-1 b_e
            acct.bytes += (sh - C64) + ncol * Vh * 3 * s64;       // bhat = b_o + kappa D_oe t
            acct.bytes += 2 * sh + ncol * Vh * (2 + 3) * s64;     // Mhat^dag bhat
            acct.launches += 4;
        } else {
            acct.bytes += ncol * (full ? 2 : 1) * Vh * 2 * s64;
            acct.launches += full ? 2 : 1;
        }
    }
    if (sys == BQ_SYS_NORMAL) {
        HIPCHK(launch_convert(PREC_F64, b_odd.all(), PREC_F64, w->bp.all(), b_odd.sites(), ncol, nullptr, 0, st));
    } else if (sys == BQ_SYS_MHAT) {
        // b' = Mhat^dag b
        CHK(k1(c64, 1, b_odd.all(), w->t64.all()));
        CHK(tv(c64, 1, 1, w->t64.all(), b_odd.all(), w->bp.all(), -kap * kap, nullptr, hw, hw));
    } else if (sys == BQ_SYS_FULL_NORMAL) {
        HIPCHK(launch_convert(PREC_F64, b_even.all(), PREC_F64, w->bp.half(0), (int)b_even.half_sites, ncol, nullptr, 0, st));
        HIPCHK(launch_convert(PREC_F64, b_odd.all(), PREC_F64, w->bp.half(1), (int)b_odd.half_sites, ncol, nullptr, 0, st));
    } else {
        // bhat = b_o + kappa D_oe T_ee^-1 b_e  (into q64),  b' = Mhat^dag bhat
        HIPCHK(launch_clover_apply(PREC_F64, op->gauge->g, op->Tinv[PREC_F64][0].p, b_even.all(), w->t64.all(), ncol, st));
        CHK(hopv(c64, 0, 1, w->t64.all(), w->q64.all(), b_odd.all(), 1.0, kap));
        CHK(k1(c64, 1, w->q64.all(), w->t64.all()));
        CHK(tv(c64, 1, 1, w->t64.all(), w->q64.all(), w->bp.all(), -kap * kap, nullptr, hw, hw));
    }

    std::vector<int> iters, nrel, status;
    if (prm.solver == BQ_SOLVER_BLOCK_CG)
        CHK(bcg_solve(op, w, prm, st, iters, nrel, status, acct));
    else
        CHK(cg_solve(op, w, prm, st, iters, nrel, status, acct));

    // final FP64 true residual of the CG system for every column
    {
        const double Vh = op->gauge->g.Vh, s64 = sp_bytes(PREC_F64);
        acct.bytes += iter_shared_bytes(op, PREC_F64) + ncol * (full ? 14 : 11) * Vh * s64;  // r = b' - A x
        acct.bytes += 2.0 * ncol * (full ? 2 : 1) * Vh * s64;                               // norms, x out
        acct.launches += 8;
        if (sys == BQ_SYS_M) {
            const double sh = stencil_shared(op, PREC_F64);
            acct.bytes += sh + ncol * Vh * 3 * s64;               // reconstruction
            acct.bytes += 2 * sh + ncol * 2 * Vh * 4 * s64;       // |b - M x|
            acct.bytes += ncol * 2 * Vh * s64;                    // |b|
            acct.launches += 7;
        }
    }
    std::vector<double> r2, b2;
    CHK(true_residual(op, w, nullptr, 0, st));
    HIPCHK(launch_fin_sum(w->partial, w->pstride, ncol, w->dtmp, st));
    r2.resize(ncol);
    HIPCHK(hipMemcpyAsync(r2.data(), w->dtmp, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    CHK(norms(op, w, w->bp, ncol, b2, st));

    // solution out
    std::vector<double> fr2(ncol, 0.0), fb2(ncol, 1.0);
    if (sys == BQ_SYS_NORMAL) {
        HIPCHK(launch_convert(PREC_F64, w->x.all(), PREC_F64, x_odd.all(), x_odd.sites(), ncol, nullptr, 0, st));
    } else if (sys == BQ_SYS_MHAT) {
        HIPCHK(launch_convert(PREC_F64, w->x.all(), PREC_F64, x_odd.all(), x_odd.sites(), ncol, nullptr, 0, st));
        // |b - Mhat x|^2 (r serves as scratch)
        CHK(k1(c64, 0, x_odd.all(), w->t64.all()));
        CHK(tvr(c64, 0, 1, w->t64.all(), x_odd.all(), b_odd.all(), w->r.all(), -kap * kap, nullptr, w->partial, hw, hw));
        HIPCHK(launch_fin_sum(w->partial, hw, ncol, w->dtmp, st));
        HIPCHK(hipMemcpyAsync(fr2.data(), w->dtmp, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        CHK(norms(op, w, b_odd, ncol, fb2, st));
    } else if (sys == BQ_SYS_FULL_NORMAL) {
        HIPCHK(launch_convert(PREC_F64, w->x.half(0), PREC_F64, x_even.all(), (int)x_even.half_sites, ncol, nullptr, 0, st));
        HIPCHK(launch_convert(PREC_F64, w->x.half(1), PREC_F64, x_odd.all(), (int)x_odd.half_sites, ncol, nullptr, 0, st));
    } else {
        HIPCHK(launch_convert(PREC_F64, w->x.all(), PREC_F64, x_odd.all(), x_odd.sites(), ncol, nullptr, 0, st));
        // x_e = T_ee^-1 (b_e + kappa D_eo x_o)
        CHK(k1(c64, 0, x_odd.all(), x_even.all(), b_even.all(), 1.0, kap));
        // |b - M x|^2 over both parities (q64 and r serve as scratch)
        CHK(tvr(c64, 0, 0, x_odd.all(), x_even.all(), b_even.all(), w->q64.all(), -kap, nullptr, w->partial, hw, 2 * hw));
        CHK(tvr(c64, 0, 1, x_even.all(), x_odd.all(), b_odd.all(), w->r.all(), -kap, nullptr, w->partial + hw, hw, 2 * hw));
        HIPCHK(launch_fin_sum(w->partial, 2 * hw, ncol, w->dtmp, st));
        HIPCHK(hipMemcpyAsync(fr2.data(), w->dtmp, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        std::vector<double> be, bo;
        CHK(norms(op, w, b_even, ncol, be, st));
        CHK(norms(op, w, b_odd, ncol, bo, st));
        for (int c2 = 0; c2 < ncol; c2++) fb2[c2] = be[c2] + bo[c2];
    }
    HIPCHK(hipStreamSynchronize(st));

    int rc = BQ_OK;
    for (int col = 0; col < ncol; col++) {
        const double tr = b2[col] > 0 ? std::sqrt(r2[col] / b2[col]) : 0.0;
        const double fr = (sys == BQ_SYS_M || sys == BQ_SYS_MHAT) ? (fb2[col] > 0 ? std::sqrt(fr2[col] / fb2[col]) : 0.0) : tr;
        int cst = BQ_OK;
        if (!std::isfinite(tr) || status[col] == COL_FAILED)
            cst = (!std::isfinite(tr) || !std::isfinite(b2[col])) ? BQ_ERR_NONFINITE : BQ_ERR_NOT_CONVERGED;
        else if (!(tr <= prm.tol))
            cst = BQ_ERR_NOT_CONVERGED;
        if (info) {
            info[col].iters = iters[col];
            info[col].reliable_updates = nrel[col];
            info[col].true_rel_resid = tr;
            info[col].full_rel_resid = fr;
            info[col].converged = cst == BQ_OK;
            info[col].status = cst;
        }
        if (cst == BQ_ERR_NONFINITE) rc = BQ_ERR_NONFINITE;
        else if (cst != BQ_OK && rc == BQ_OK) rc = cst;
    }
    if (rc == BQ_ERR_NOT_CONVERGED) fail(rc, "some right-hand side did not converge within maxiter");
    if (rc == BQ_ERR_NONFINITE) fail(rc, "non-finite value in the source or during the solve");
    return rc;
}

// ---------------------------------------------------------------------------
// BiCGstab on Mhat (the solver list's BiCGstab), van der Vorst's recursion per column in the
// inner precision with FP64 reductions.  Mhat is not Hermitian at mu != 0, and BiCGstab works
// on Mhat itself instead of the normal equations.  An inner run stops when its recursive
// residual falls below delta times the last FP64 residual (or reaches tol |bhat|); the FP64
// residual bhat - Mhat x is then recomputed, and the column is done or restarts from it.
// ---------------------------------------------------------------------------

static int bicg_views(bq_op op, const Vec& b_even, const Vec& b_odd, const Vec& x_even, const Vec& x_odd, int ncol,
                      const bq_solve_params& prm, bq_solve_info* info, hipStream_t st, SolveAcct& acct)
{
    const int sys = prm.system;
    const int prec = prm.inner_prec;
    bq_context ctx = op->gauge->ctx;
    const Geom& g = op->gauge->g;
    const double kap = op->kappa;
    const int hw = pad_sites(g.Vh) / kTile;
    // workspace: FP64 bhat, x64, r64, odd q64 and even t64 scratch; inner r, rhat, p, v, s, t, even te, x
    DevBuf d[16], sc[16];
    Vec bh, x64, r64, q64, t64, r, rh, p, v, s_, t, te, xi;
    int k = 0;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[k], sc[k], bh)); k++;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[k], sc[k], x64)); k++;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[k], sc[k], r64)); k++;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[k], sc[k], q64)); k++;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, d[k], sc[k], t64)); k++;
    for (Vec* vv : {&r, &rh, &p, &v, &s_, &t, &te}) {
        CHK(alloc_vec(ctx, g, prec, 1, ncol, d[k], sc[k], *vv));
        k++;
    }
    if (prec == PREC_F64) xi = x64;
    else CHK(alloc_vec(ctx, g, prec, 1, ncol, d[k], sc[k], xi));
    const int n = (int)bh.half_sites;
    DevBuf part, scal, ints;
    CHK(part.alloc(ctx, sizeof(double) * (size_t)hw * ncol * 4));
    CHK(scal.alloc(ctx, sizeof(double) * (size_t)ncol * 11));
    CHK(ints.alloc(ctx, sizeof(int) * (size_t)ncol * 4));
    double* pt = part.as<double>();
    BicgScalars S{};
    {
        double* q = scal.as<double>();
        S.rho = (double2*)q; S.alpha = (double2*)(q + 2 * ncol); S.omega = (double2*)(q + 4 * ncol);
        S.beta = (double2*)(q + 6 * ncol); S.r2 = q + 8 * ncol; S.stop2 = q + 9 * ncol; S.tol2b2 = q + 10 * ncol;
        int* i = ints.as<int>();
        S.status = i; S.iters = i + ncol; S.nrel = i + 2 * ncol; S.restart = i + 3 * ncol;
        const double delta = prm.delta > 0 ? prm.delta : (prec == PREC_F32 ? 0.01 : 0.0);
        S.delta2 = delta * delta;
    }
    OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, nullptr, 1, st};
    const double s64 = sp_bytes(PREC_F64), sP = sp_bytes(prec), Vh = g.Vh;
    // bhat
    if (sys == BQ_SYS_M) {
        HIPCHK(launch_clover_apply(PREC_F64, g, op->Tinv[PREC_F64][0].p, b_even.all(), t64.all(), ncol, st));
        CHK(hopv(c64, 0, 1, t64.all(), bh.all(), b_odd.all(), 1.0, kap));
        acct.bytes += stencil_shared(op, PREC_F64) + ncol * Vh * 5 * s64;
    } else {
        HIPCHK(launch_convert(PREC_F64, b_odd.all(), PREC_F64, bh.all(), n, ncol, nullptr, 0, st));
        acct.bytes += ncol * Vh * 2 * s64;
    }
    // start: x = 0, r64 = bhat, every column "stopped" so that the first reliable pass sets it up
    std::vector<double> b2(ncol), t2(ncol);
    HIPCHK(launch_norm2(PREC_F64, bh.all(), n, ncol, pt, hw, st));
    HIPCHK(launch_fin_sum(pt, hw, ncol, S.r2, st));
    HIPCHK(hipMemcpyAsync(b2.data(), S.r2, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < ncol; c++) t2[c] = prm.tol * prm.tol * b2[c];
    HIPCHK(hipMemcpyAsync(S.tol2b2, t2.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, st));
    {
        std::vector<int> z(4 * ncol, 0);
        for (int c = 0; c < ncol; c++) z[c] = COL_STOPPED;
        HIPCHK(hipMemcpyAsync(S.status, z.data(), sizeof(int) * 4 * ncol, hipMemcpyHostToDevice, st));
    }
    HIPCHK(launch_zero(PREC_F64, x64.all(), n, ncol, nullptr, 0, st));
    HIPCHK(launch_convert(PREC_F64, bh.all(), PREC_F64, r64.all(), n, ncol, nullptr, 0, st));
    const int mRestart = 1 << COL_JUST_STOPPED, mStopped = 1 << COL_STOPPED;
    // decide / restart: partials of |r64|^2 are in pt
    auto restart = [&]() -> int {
        HIPCHK(launch_fin_bicg(3, S, pt, hw, ncol, st));
        if (prec != PREC_F64) HIPCHK(launch_zero(prec, xi.all(), n, ncol, S.status, mRestart, st));
        HIPCHK(launch_convert(PREC_F64, r64.all(), prec, r.all(), n, ncol, S.status, mRestart, st));
        HIPCHK(launch_convert(prec, r.all(), prec, rh.all(), n, ncol, S.status, mRestart, st));
        HIPCHK(launch_zero(prec, p.all(), n, ncol, S.status, mRestart, st));
        HIPCHK(launch_zero(prec, v.all(), n, ncol, S.status, mRestart, st));
        HIPCHK(launch_set_status(S.status, S.restart, ncol, COL_ACTIVE, st));
        return BQ_OK;
    };
    HIPCHK(launch_norm2(PREC_F64, r64.all(), n, ncol, pt, hw, st));
    CHK(restart());
    const int kchunk = prm.chunk > 0 ? prm.chunk : 4;
    const long maxiter = prm.maxiter > 0 ? prm.maxiter : 100000;
    OpCall ci{op, prec, get_tune(ctx, prec, ncol), ncol, S.status, 1 << COL_ACTIVE, st};
    OpCall cr{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, S.status, mStopped, st};
    std::vector<int> hs(3 * ncol), prev(3 * ncol, 0);
    long done = 0;
    const double ishared = 4 * stencil_shared(op, prec), icol = Vh * 30 * sP;
    const double rshared = 2 * stencil_shared(op, PREC_F64), rcol = Vh * (7 * s64 + (prec != PREC_F64 ? 2 * (s64 + sP) : 0));
    while (true) {
        for (int it = 0; it < kchunk; it++) {
            HIPCHK(launch_bicg_p(prec, r.all(), p.all(), v.all(), S, n, ncol, st));
            CHK(k1(ci, 0, p.all(), te.all()));
            CHK(tv(ci, 0, 1, te.all(), p.all(), v.all(), -kap * kap, nullptr, hw, hw));
            HIPCHK(launch_dots2(prec, rh.all(), v.all(), FieldArg(), FieldArg(), S.status, n, ncol, pt, hw, st));
            HIPCHK(launch_fin_bicg(0, S, pt, hw, ncol, st));
            HIPCHK(launch_bicg_s(prec, r.all(), v.all(), s_.all(), S, n, ncol, st));
            CHK(k1(ci, 0, s_.all(), te.all()));
            CHK(tv(ci, 0, 1, te.all(), s_.all(), t.all(), -kap * kap, nullptr, hw, hw));
            HIPCHK(launch_dots2(prec, t.all(), s_.all(), t.all(), t.all(), S.status, n, ncol, pt, hw, st));
            HIPCHK(launch_fin_bicg(1, S, pt, hw, ncol, st));
            HIPCHK(launch_bicg_xr(prec, xi.all(), p.all(), s_.all(), t.all(), r.all(), rh.all(), S, n, ncol, pt, hw, st));
            HIPCHK(launch_fin_bicg(2, S, pt, hw, ncol, st));
        }
        // reliable pass for the columns whose inner run stopped: x64 += x, r64 = bhat - Mhat x64
        if (prec != PREC_F64) HIPCHK(launch_accum(prec, xi.all(), x64.all(), n, ncol, S.status, mStopped, st));
        CHK(k1(cr, 0, x64.all(), t64.all()));
        CHK(tvr(cr, 0, 1, t64.all(), x64.all(), bh.all(), r64.all(), -kap * kap, nullptr, pt, hw, hw));
        CHK(restart());
        done += kchunk;
        acct.chunks++;
        acct.iterations += kchunk;
        acct.launches += 12L * kchunk + 9 + (prec != PREC_F64);
        HIPCHK(hipMemcpyAsync(hs.data(), S.status, sizeof(int) * 3 * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int dmax = 0, nrel = 0;
        double colit = 0;
        for (int c = 0; c < ncol; c++) {
            const int di = hs[ncol + c] - prev[ncol + c];
            dmax = std::max(dmax, di);
            colit += di;
            nrel += hs[2 * ncol + c] - prev[2 * ncol + c];
        }
        acct.bytes += dmax * ishared + colit * icol + (nrel > 0 ? rshared + nrel * rcol : 0.0);
        prev = hs;
        bool all = true;
        for (int c = 0; c < ncol; c++)
            if (hs[c] != COL_DONE && hs[c] != COL_FAILED) all = false;
        if (all || done >= maxiter) break;
    }
    // columns still iterating: fold the inner iterate
    if (prec != PREC_F64)
        HIPCHK(launch_accum(prec, xi.all(), x64.all(), n, ncol, S.status, (1 << COL_ACTIVE) | mStopped, st));
    // final FP64 residual |bhat - Mhat x| for every column
    CHK(k1(c64, 0, x64.all(), t64.all()));
    CHK(tvr(c64, 0, 1, t64.all(), x64.all(), bh.all(), r64.all(), -kap * kap, nullptr, pt, hw, hw));
    std::vector<double> r2(ncol), fr2(ncol, 0.0), fb2(ncol, 1.0);
    HIPCHK(launch_fin_sum(pt, hw, ncol, S.r2, st));
    HIPCHK(hipMemcpyAsync(r2.data(), S.r2, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(launch_convert(PREC_F64, x64.all(), PREC_F64, x_odd.all(), n, ncol, nullptr, 0, st));
    acct.bytes += rshared + ncol * Vh * 9 * s64;
    if (sys == BQ_SYS_M) {
        // x_e = T_ee^-1 (b_e + kappa D_eo x_o); |b - M x|^2 over both parities
        CHK(k1(c64, 0, x_odd.all(), x_even.all(), b_even.all(), 1.0, kap));
        CHK(tvr(c64, 0, 0, x_odd.all(), x_even.all(), b_even.all(), t64.all(), -kap, nullptr, pt, hw, 2 * hw));
        CHK(tvr(c64, 0, 1, x_even.all(), x_odd.all(), b_odd.all(), q64.all(), -kap, nullptr, pt + hw, hw, 2 * hw));
        HIPCHK(launch_fin_sum(pt, 2 * hw, ncol, S.r2, st));
        HIPCHK(hipMemcpyAsync(fr2.data(), S.r2, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(launch_norm2(PREC_F64, b_even.all(), n, ncol, pt, hw, st));
        HIPCHK(launch_norm2(PREC_F64, b_odd.all(), n, ncol, pt + (size_t)hw * ncol, hw, st));
        HIPCHK(launch_fin_sum(pt, hw, 2 * ncol, S.stop2, st));
        std::vector<double> be(2 * ncol);
        HIPCHK(hipMemcpyAsync(be.data(), S.stop2, sizeof(double) * 2 * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int c = 0; c < ncol; c++) fb2[c] = be[c] + be[ncol + c];
        acct.bytes += 3 * stencil_shared(op, PREC_F64) + ncol * Vh * 13 * s64;
    }
    std::vector<int> h(3 * ncol);
    HIPCHK(hipMemcpyAsync(h.data(), S.status, sizeof(int) * 3 * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int rc = BQ_OK;
    for (int c = 0; c < ncol; c++) {
        const double tr = b2[c] > 0 ? std::sqrt(r2[c] / b2[c]) : 0.0;
        const double fr = sys == BQ_SYS_M ? (fb2[c] > 0 ? std::sqrt(fr2[c] / fb2[c]) : 0.0) : tr;
        int cst = BQ_OK;
        if (!std::isfinite(tr)) cst = BQ_ERR_NONFINITE;
        else if (h[c] == COL_FAILED || !(tr <= prm.tol)) cst = BQ_ERR_NOT_CONVERGED;
        if (info) {
            info[c].iters = h[ncol + c];
            info[c].reliable_updates = std::max(0, h[2 * ncol + c] - 1);  // the first pass only sets up
            info[c].true_rel_resid = tr;
            info[c].full_rel_resid = fr;
            info[c].converged = cst == BQ_OK;
            info[c].status = cst;
        }
        if (cst == BQ_ERR_NONFINITE) rc = cst;
        else if (cst != BQ_OK && rc == BQ_OK) rc = cst;
    }
    if (rc == BQ_ERR_NOT_CONVERGED) fail(rc, "some right-hand side did not converge within maxiter");
    if (rc == BQ_ERR_NONFINITE) fail(rc, "non-finite value in the source or during the solve");
    return rc;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int bq_version(void) { return 10000; }

const char* bq_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// static work memory of the allocation-free apply
// ---------------------------------------------------------------------------

// One copy per device, loaded with the library's code object and held until the process ends.
// Host code never uses this name as an address (on the host it only stands for the symbol): the
// device address of each device's copy comes from hipGetSymbolAddress, taken once per device at
// context creation and kept in scratch_base.
static __device__ __align__(256) unsigned char scratch[BQ_NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static std::vector<void*> scratch_base;  // per device ordinal

// Take the address of the current device's copy of `scratch` (device `device` must be current).
static int scratch_resolve(int device)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    if ((int)scratch_base.size() <= device) scratch_base.resize(device + 1, nullptr);
    if (scratch_base[device]) return BQ_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(BQ_ERR_DEVICE, "no device address for the static work array on device %d: %s", device,
                    hipGetErrorString(e));
    scratch_base[device] = p;
    return BQ_OK;
}

static void* scratch_on(int device)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    return device < (int)scratch_base.size() ? scratch_base[device] : nullptr;
}

int bq_context_create(int device, uint64_t hbm_budget_bytes, bq_alloc_fn alloc, bq_dealloc_fn dealloc,
                      void* alloc_ctx, bq_context* out)
{
    if (!out) return fail(BQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if ((alloc == nullptr) != (dealloc == nullptr))
        return fail(BQ_ERR_INVALID, "alloc and dealloc must both be given or both be NULL");
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(BQ_ERR_INVALID, "device %d out of range (%d devices)", device, n);
    HIPCHK(hipSetDevice(device));
    CHK(scratch_resolve(device));
    auto c = std::make_unique<bq_context_s>();
    c->device = device;
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
    c->alloc = alloc;
    c->dealloc = dealloc;
    c->alloc_ctx = alloc_ctx;
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    *out = c.release();
    return BQ_OK;
}

int bq_context_destroy(bq_context ctx)
{
    if (!ctx) return BQ_OK;
    if (ctx->closing) return fail(BQ_ERR_INVALID, "context already destroyed");
    if (ctx->nhandles > 0) {  // freed together with its last handle
        ctx->closing = true;
        return BQ_OK;
    }
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return BQ_OK;
}

int bq_context_hbm_used(bq_context ctx, uint64_t* used)
{
    if (!ctx || !used) return fail(BQ_ERR_INVALID, "NULL argument");
    *used = ctx->used;
    return BQ_OK;
}

int bq_gauge_upload(bq_context ctx, const int dims[4], const double* links, int links_on_device, int t_bc,
                    bq_gauge* out)
{
    if (!ctx || !links || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (!dims_ok(dims)) return fail(BQ_ERR_INVALID, "lattice extents must be even, >= 2, with V/2 < 2^24");
    if (t_bc != 1 && t_bc != -1) return fail(BQ_ERR_INVALID, "t_bc must be +1 or -1");
    HIPCHK(hipSetDevice(ctx->device));
    auto G = std::make_unique<bq_gauge_s>();
    G->ctx = ctx;
    std::memcpy(G->dims, dims, sizeof(G->dims));
    G->g = make_geom(dims);
    G->t_bc = t_bc;
    const size_t V = 2 * (size_t)G->g.Vh;
    const size_t nbytes = 4 * V * 9 * 16;
    DevBuf stage;
    const double2* canon = (const double2*)links;
    if (!links_on_device) {
        CHK(stage.alloc(ctx, nbytes));
        HIPCHK(hipMemcpyAsync(stage.p, links, nbytes, hipMemcpyHostToDevice, ctx->stream));
        canon = stage.as<double2>();
    }
    // The two-row link form rebuilds row 2 as conj(row0 x row1), which holds for SU(3) only: it is
    // kept for a storage precision only if every link is SU(3) to well within that precision's
    // rounding.  Without it FP64 and FP32 stencils read all 18 reals, and FP16 storage and the
    // server (both two-row only) report BQ_ERR_UNSUPPORTED.
    {
        const size_t nl = 4 * V;
        const int np = link_su3_parts(nl);
        DevBuf part;
        CHK(part.alloc(ctx, sizeof(double) * np));
        HIPCHK(launch_link_su3_dev(canon, nl, part.as<double>(), ctx->stream));
        std::vector<double> h(np);
        HIPCHK(hipMemcpyAsync(h.data(), part.p, sizeof(double) * np, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        double d = 0;
        for (double v : h) d = std::isnan(v) ? INFINITY : std::max(d, v);
        G->su3_dev = d;
        if (!std::isfinite(d)) return fail(BQ_ERR_NONFINITE, "non-finite gauge link");
    }
    const int forms[5][2] = {{PREC_F64, 18}, {PREC_F64, 12}, {PREC_F32, 18}, {PREC_F32, 12}, {PREC_F16, 12}};
    const size_t Vp = pad_sites(G->g.Vh);
    for (int f = 0; f < 5; f++) {
        LinkSet& ls = G->links[f];
        if (forms[f][1] == 12 && G->su3_dev > su3_tolerance(forms[f][0])) continue;
        ls.prec = forms[f][0];
        ls.recon = forms[f][1];
        const size_t per = Vp * link_nu(ls.prec, ls.recon) * unit_bytes(ls.prec) + kSkew;
        CHK(ls.buf.alloc(ctx, per * 8));
        for (int k = 0; k < 8; k++) ls.U[k] = (char*)ls.buf.p + per * k;
        for (int p = 0; p < 2; p++) {
            void* dst[4] = {(void*)ls.U[p * 4 + 0], (void*)ls.U[p * 4 + 1], (void*)ls.U[p * 4 + 2], (void*)ls.U[p * 4 + 3]};
            HIPCHK(launch_links_import(canon, G->g, p, ls.prec, ls.recon, dst, ctx->stream));
        }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = G.release();
    ctx->nhandles++;
    return BQ_OK;
}

int bq_gauge_su3_deviation(bq_gauge g, double* dev)
{
    if (!g || !dev) return fail(BQ_ERR_INVALID, "NULL argument");
    *dev = g->su3_dev;
    return BQ_OK;
}

int bq_gauge_plaquette(bq_gauge g, double* plaq)
{
    if (!g || !plaq) return fail(BQ_ERR_INVALID, "NULL argument");
    bq_context ctx = g->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const int nw = pad_sites(g->g.Vh) / kTile;
    DevBuf part;
    CHK(part.alloc(ctx, sizeof(double) * 2 * nw));
    const LinkSet* ls = g->get(PREC_F64, 18);
    const double2* U[8];
    for (int k = 0; k < 8; k++) U[k] = (const double2*)ls->U[k];
    HIPCHK(launch_plaquette(g->g, U, part.as<double>(), 2 * nw, ctx->stream));
    std::vector<double> h(2 * nw);
    HIPCHK(hipMemcpyAsync(h.data(), part.p, sizeof(double) * 2 * nw, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double s = 0;
    for (double v : h) s += v;
    *plaq = s / (6.0 * 2.0 * g->g.Vh);
    return BQ_OK;
}

int bq_gauge_free(bq_gauge g)
{
    if (!g) return BQ_OK;
    if (g->nops > 0) return fail(BQ_ERR_BUSY, "%d operator(s) still use this gauge field", g->nops);
    if (g->nsess > 0)
        return fail(BQ_ERR_BUSY, "%d server session(s) still hold this gauge field (bq_server_release)", g->nsess);
    bq_context ctx = g->ctx;
    (void)hipSetDevice(ctx->device);
    delete g;
    ctx_release_handle(ctx);
    return BQ_OK;
}

}  // extern "C"

// Operator construction.  The gauge field keeps B = sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}
// (independent of kappa and c_SW), built once from the links; an operator then needs only
// T = 1 + kappa c_SW B and the Cholesky inverse of its blocks.
// lean_prec >= 0 builds only what a solve in that inner precision needs: FP64 T on both
// parities and T_ee^-1, plus T_oo and T_ee^-1 in lean_prec.
// The clover arrays of an operator for kappa and c_SW from the gauge field's kappa-independent B
// (Eq. 2), into arrays op_build allocated for the same lean precision, on stream st; then waits
// for st.  flag: one device int for the positive-definiteness check.
static int clover_fill(bq_op op, double kappa, double csw, int lean_prec, int* flag, hipStream_t st)
{
    bq_gauge g = op->gauge;
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
    for (int p = 0; p < 2; p++) {
        const bool inv = lean_prec < 0 || p == 0;
        HIPCHK(launch_clover_from_B(g->g, p, g->B[p].as<double2>(), kappa * csw, op->T[PREC_F64][p].as<double2>(),
                                    inv ? op->Tinv[PREC_F64][p].as<double2>() : nullptr, flag, st));
    }
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hbad) return fail(BQ_ERR_CLOVER_NOT_HPD, "clover block not positive definite (kappa*c_SW = %g)", kappa * csw);
    for (int prec : {PREC_F32, PREC_F16}) {
        if (lean_prec >= 0 && prec != lean_prec) continue;
        for (int p = 0; p < 2; p++) {
            if (lean_prec < 0 || p == 1)
                HIPCHK(launch_clover_convert(prec, op->T[PREC_F64][p].as<double2>(), op->T[prec][p].p, g->g.Vh, st));
            if (lean_prec < 0 || p == 0)
                HIPCHK(launch_clover_convert(prec, op->Tinv[PREC_F64][p].as<double2>(), op->Tinv[prec][p].p, g->g.Vh,
                                             st));
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    op->kappa = kappa;
    op->csw = csw;
    return BQ_OK;
}

// flag, st: a device int for the positive-definiteness check and the stream to build on (a server
// session's); NULL: a flag of its own and the context stream.
static int op_build(bq_gauge g, double kappa, double csw, double mu, int lean_prec, bq_op* out,
                    int* flag = nullptr, hipStream_t st = nullptr)
{
    if (!g || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (!std::isfinite(kappa) || !std::isfinite(csw) || !std::isfinite(mu))
        return fail(BQ_ERR_INVALID, "kappa, c_SW and mu must be finite");
    bq_context ctx = g->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const size_t Vp = pad_sites(g->g.Vh);
    if (!g->B[0].p) {
        for (int p = 0; p < 2; p++) CHK(g->B[p].alloc(ctx, Vp * 36 * 16));
        CloverBuild cb;
        cb.g = g->g;
        const LinkSet* ls = g->get(PREC_F64, 18);
        for (int k = 0; k < 8; k++) cb.U64[k] = (const double2*)ls->U[k];
        for (int p = 0; p < 2; p++) cb.B[p] = g->B[p].as<double2>();
        HIPCHK(launch_clover_build(cb, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));  // B is read on the build stream below
    }
    auto op = std::make_unique<bq_op_s>();
    op->gauge = g;
    op->mu = mu;
    for (int p = 0; p < 2; p++) {
        CHK(op->T[PREC_F64][p].alloc(ctx, Vp * 36 * 16));
        if (lean_prec < 0 || p == 0) CHK(op->Tinv[PREC_F64][p].alloc(ctx, Vp * 36 * 16));
    }
    for (int prec : {PREC_F32, PREC_F16}) {
        if (lean_prec >= 0 && prec != lean_prec) continue;
        const size_t bytes = Vp * clover_nu(prec) * unit_bytes(prec);
        for (int p = 0; p < 2; p++) {
            if (lean_prec < 0 || p == 1) CHK(op->T[prec][p].alloc(ctx, bytes));
            if (lean_prec < 0 || p == 0) CHK(op->Tinv[prec][p].alloc(ctx, bytes));
        }
    }
    DevBuf own;
    if (!flag) {
        CHK(own.alloc(ctx, sizeof(int)));
        flag = own.as<int>();
    }
    g->nops++;  // from here the operator is whole: freeing it releases this count
    bq_op o = op.release();
    const int rc = clover_fill(o, kappa, csw, lean_prec, flag, st ? st : ctx->stream);
    if (rc != BQ_OK) {
        bq_op_free(o);
        return rc;
    }
    *out = o;
    return BQ_OK;
}

extern "C" {

int bq_op_create(bq_gauge g, double kappa, double csw, double mu, bq_op* out)
{
    return op_build(g, kappa, csw, mu, -1, out);
}

int bq_op_free(bq_op op)
{
    if (!op) return BQ_OK;
    (void)hipSetDevice(op->gauge->ctx->device);
    op->gauge->nops--;
    delete op;
    return BQ_OK;
}

int bq_field_create(bq_context ctx, const int dims[4], int subset, int prec, int nrhs, bq_field* out)
{
    if (!ctx || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (!dims_ok(dims)) return fail(BQ_ERR_INVALID, "lattice extents must be even, >= 2, with V/2 < 2^24");
    if (subset < BQ_EVEN || subset > BQ_FULL) return fail(BQ_ERR_INVALID, "bad subset %d", subset);
    if (prec < BQ_F64 || prec > BQ_F16) return fail(BQ_ERR_INVALID, "bad precision %d", prec);
    if (nrhs < 1) return fail(BQ_ERR_INVALID, "nrhs must be >= 1");
    HIPCHK(hipSetDevice(ctx->device));
    auto f = std::make_unique<bq_field_s>();
    f->ctx = ctx;
    std::memcpy(f->dims, dims, sizeof(f->dims));
    f->g = make_geom(dims);
    f->subset = subset;
    f->prec = prec;
    f->nrhs = nrhs;
    f->nh = subset == BQ_FULL ? 2 : 1;
    f->half_sites = pad_sites(f->g.Vh);
    f->half_units = f->half_sites * spinor_nu(prec);
    f->cstride = f->half_units * f->nh + col_pad_units(prec);
    f->sstride = f->half_sites * f->nh + col_pad_scales();
    CHK(f->data.alloc(ctx, f->cstride * nrhs * unit_bytes(prec)));
    if (prec == BQ_F16) CHK(f->scale.alloc(ctx, f->sstride * nrhs * sizeof(float)));
    *out = f.release();
    ctx->nhandles++;
    return BQ_OK;
}

int bq_field_free(bq_field f)
{
    if (!f) return BQ_OK;
    bq_context ctx = f->ctx;
    (void)hipSetDevice(ctx->device);
    delete f;
    ctx_release_handle(ctx);
    return BQ_OK;
}

static void field_parities(bq_field f, int* p0, int* p1)
{
    *p0 = f->subset == BQ_ODD ? 1 : 0;
    *p1 = f->subset == BQ_EVEN ? 0 : 1;
}

int bq_field_put(bq_field f, const double* src, int src_on_device, void* stream)
{
    if (!f || !src) return fail(BQ_ERR_INVALID, "NULL argument");
    bq_context ctx = f->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    CHK(sync_with(ctx, (hipStream_t)stream));
    const size_t bytes = (size_t)f->nrhs * 2 * f->g.Vh * 12 * 16;
    DevBuf stage;
    const double2* canon = (const double2*)src;
    if (!src_on_device) {
        CHK(stage.alloc(ctx, bytes));
        HIPCHK(hipMemcpyAsync(stage.p, src, bytes, hipMemcpyHostToDevice, ctx->stream));
        canon = stage.as<double2>();
    }
    int p0, p1;
    field_parities(f, &p0, &p1);
    for (int p = p0; p <= p1; p++) {
        Vec v = parity_vec(f, p);
        HIPCHK(launch_spinor_import(canon, f->nrhs, f->g, p, f->prec, v.all(), ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BQ_OK;
}

int bq_field_get(bq_field f, double* dst, int dst_on_device, void* stream)
{
    if (!f || !dst) return fail(BQ_ERR_INVALID, "NULL argument");
    bq_context ctx = f->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    CHK(sync_with(ctx, (hipStream_t)stream));
    const size_t bytes = (size_t)f->nrhs * 2 * f->g.Vh * 12 * 16;
    DevBuf stage;
    double2* canon = (double2*)dst;
    if (!dst_on_device) {
        CHK(stage.alloc(ctx, bytes));
        // keep the sites outside the field's subset as the caller had them
        if (f->subset != BQ_FULL) HIPCHK(hipMemcpyAsync(stage.p, dst, bytes, hipMemcpyHostToDevice, ctx->stream));
        canon = stage.as<double2>();
    }
    int p0, p1;
    field_parities(f, &p0, &p1);
    for (int p = p0; p <= p1; p++) {
        Vec v = parity_vec(f, p);
        HIPCHK(launch_spinor_export(v.all(), f->nrhs, f->g, p, f->prec, canon, ctx->stream));
    }
    if (!dst_on_device) HIPCHK(hipMemcpyAsync(dst, stage.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BQ_OK;
}

// fields the library creates for its own use are released through the ABI call (handle count)
struct FieldFree {
    void operator()(bq_field f) const { (void)bq_field_free(f); }
};
using FieldPtr = std::unique_ptr<bq_field_s, FieldFree>;

// required subsets per kind: {in, out}
static bool kind_subsets(int kind, int* in, int* out)
{
    switch (kind) {
    case BQ_OP_M: case BQ_OP_MDAG: case BQ_OP_CLOVER: case BQ_OP_MDAGM: *in = BQ_FULL; *out = BQ_FULL; return true;
    case BQ_OP_MHAT: case BQ_OP_MHATDAG: case BQ_OP_MHATDAG_MHAT: *in = BQ_ODD; *out = BQ_ODD; return true;
    case BQ_OP_DEO: case BQ_OP_DEO_DAG: case BQ_OP_K1: case BQ_OP_K1_DAG: *in = BQ_ODD; *out = BQ_EVEN; return true;
    case BQ_OP_DOE: case BQ_OP_DOE_DAG: *in = BQ_EVEN; *out = BQ_ODD; return true;
    case BQ_OP_CLOVER_INV: *in = BQ_EVEN; *out = BQ_EVEN; return true;
    }
    return false;
}

struct Scratch {
    DevBuf d1, s1, d2, s2;
    Vec a, b;
};

static int apply_impl(bq_op op, int kind, bq_field in, bq_field out, hipStream_t st, Scratch& scr)
{
    bq_context ctx = op->gauge->ctx;
    const int prec = in->prec, ncol = in->nrhs;
    const double k = op->kappa;
    OpCall c{op, prec, get_tune(ctx, prec, ncol), ncol, nullptr, 1, st};
    const Geom& g = op->gauge->g;
    switch (kind) {
    case BQ_OP_M:
    case BQ_OP_MDAG: {
        const int dag = kind == BQ_OP_MDAG;
        Vec ie = parity_vec(in, 0), io = parity_vec(in, 1), oe = parity_vec(out, 0), oo = parity_vec(out, 1);
        CHK(tv(c, dag, 0, io.all(), ie.all(), oe.all(), -k, nullptr, 0, 0));
        return tv(c, dag, 1, ie.all(), io.all(), oo.all(), -k, nullptr, 0, 0);
    }
    case BQ_OP_MDAGM: {
        if (!scr.a.d) CHK(alloc_vec(ctx, g, prec, 2, ncol, scr.d1, scr.s1, scr.a));
        Vec ie = parity_vec(in, 0), io = parity_vec(in, 1), oe = parity_vec(out, 0), oo = parity_vec(out, 1);
        CHK(tv(c, 0, 0, io.all(), ie.all(), scr.a.half(0), -k, nullptr, 0, 0));
        CHK(tv(c, 0, 1, ie.all(), io.all(), scr.a.half(1), -k, nullptr, 0, 0));
        CHK(tv(c, 1, 0, scr.a.half(1), scr.a.half(0), oe.all(), -k, nullptr, 0, 0));
        return tv(c, 1, 1, scr.a.half(0), scr.a.half(1), oo.all(), -k, nullptr, 0, 0);
    }
    case BQ_OP_MHAT:
    case BQ_OP_MHATDAG: {
        const int dag = kind == BQ_OP_MHATDAG;
        if (!scr.a.d) CHK(alloc_vec(ctx, g, prec, 1, ncol, scr.d1, scr.s1, scr.a));
        Vec io = parity_vec(in, 1), oo = parity_vec(out, 1);
        CHK(k1(c, dag, io.all(), scr.a.all()));
        return tv(c, dag, 1, scr.a.all(), io.all(), oo.all(), -k * k, nullptr, 0, 0);
    }
    case BQ_OP_MHATDAG_MHAT: {
        if (!scr.a.d) CHK(alloc_vec(ctx, g, prec, 1, ncol, scr.d1, scr.s1, scr.a));
        if (!scr.b.d) CHK(alloc_vec(ctx, g, prec, 1, ncol, scr.d2, scr.s2, scr.b));
        Vec io = parity_vec(in, 1), oo = parity_vec(out, 1);
        CHK(k1(c, 0, io.all(), scr.a.all()));
        CHK(tv(c, 0, 1, scr.a.all(), io.all(), scr.b.all(), -k * k, nullptr, 0, 0));
        CHK(k1(c, 1, scr.b.all(), scr.a.all()));
        return tv(c, 1, 1, scr.a.all(), scr.b.all(), oo.all(), -k * k, nullptr, 0, 0);
    }
    case BQ_OP_DEO:
    case BQ_OP_DEO_DAG:
        return hopv(c, kind == BQ_OP_DEO_DAG, 0, parity_vec(in, 1).all(), parity_vec(out, 0).all(), FieldArg(), 0, 1);
    case BQ_OP_DOE:
    case BQ_OP_DOE_DAG:
        return hopv(c, kind == BQ_OP_DOE_DAG, 1, parity_vec(in, 0).all(), parity_vec(out, 1).all(), FieldArg(), 0, 1);
    case BQ_OP_K1:
    case BQ_OP_K1_DAG:
        return k1(c, kind == BQ_OP_K1_DAG, parity_vec(in, 1).all(), parity_vec(out, 0).all());
    case BQ_OP_CLOVER:
        for (int p = 0; p < 2; p++)
            HIPCHK(launch_clover_apply(prec, g, op->T[prec][p].p, parity_vec(in, p).all(), parity_vec(out, p).all(), ncol, st));
        return BQ_OK;
    case BQ_OP_CLOVER_INV:
        HIPCHK(launch_clover_apply(prec, g, op->Tinv[prec][0].p, parity_vec(in, 0).all(), parity_vec(out, 0).all(), ncol, st));
        return BQ_OK;
    }
    return fail(BQ_ERR_INVALID, "unknown operator kind %d", kind);
}

static int apply_check(bq_op op, int kind, bq_field in, bq_field out)
{
    if (!op || !in || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    int si, so;
    if (!kind_subsets(kind, &si, &so)) return fail(BQ_ERR_INVALID, "unknown operator kind %d", kind);
    if (in->subset != si || out->subset != so)
        return fail(BQ_ERR_INVALID, "operator %d needs subsets (%d -> %d), got (%d -> %d)", kind, si, so, in->subset,
                    out->subset);
    if (in->prec != out->prec || in->nrhs != out->nrhs) return fail(BQ_ERR_INVALID, "in/out precision or nrhs differ");
    if (in == out) return fail(BQ_ERR_INVALID, "in and out must be different fields");
    for (int k = 0; k < 4; k++)
        if (in->dims[k] != op->gauge->dims[k] || out->dims[k] != op->gauge->dims[k])
            return fail(BQ_ERR_INVALID, "field and gauge lattices differ");
    return BQ_OK;
}

int bq_apply(bq_op op, int kind, bq_field in, bq_field out, void* stream)
{
    CHK(apply_check(op, kind, in, out));
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    Scratch scr;
    int rc = apply_impl(op, kind, in, out, st, scr);
    if (scr.a.d || scr.b.d) HIPCHK(hipStreamSynchronize(st));  // scratch is freed on return
    return rc;
}

// Work fields apply_impl needs for an operator kind: how many, and of how many halves.
static void apply_work_fields(int kind, int& n, int& nh)
{
    n = 0;
    nh = 1;
    switch (kind) {
    case BQ_OP_MDAGM: n = 1; nh = 2; break;
    case BQ_OP_MHAT: case BQ_OP_MHATDAG: n = 1; break;
    case BQ_OP_MHATDAG_MHAT: n = 2; break;
    }
}

int bq_apply_noalloc(bq_op op, int kind, bq_field in, bq_field out, void* stream)
{
    CHK(apply_check(op, kind, in, out));
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    char* base = (char*)scratch_on(ctx->device);
    if (!base) return fail(BQ_ERR_DEVICE, "static work array of device %d not resolved", ctx->device);
    int n = 0, nh = 1;
    apply_work_fields(kind, n, nh);
    // the work fields one after the other, each array on a 256-byte boundary
    Scratch scr;
    Vec* v[2] = {&scr.a, &scr.b};
    size_t at[2][2] = {}, end = 0;
    for (int i = 0; i < n; i++) {
        size_t db = 0, sb = 0;
        vec_layout(op->gauge->g, in->prec, nh, in->nrhs, *v[i], db, sb);
        at[i][0] = end;
        end += (db + 255) & ~(size_t)255;
        at[i][1] = end;
        end += (sb + 255) & ~(size_t)255;
    }
    if (end > (size_t)BQ_NOALLOC_SCRATCH_BYTES)
        return fail(BQ_ERR_INVALID,
                    "operator kind %d with %d columns on this lattice needs %zu bytes of work fields; the "
                    "allocation-free apply has %llu",
                    kind, in->nrhs, end, (unsigned long long)BQ_NOALLOC_SCRATCH_BYTES);
    for (int i = 0; i < n; i++) {
        v[i]->d = base + at[i][0];
        v[i]->s = in->prec == PREC_F16 ? (float*)(base + at[i][1]) : nullptr;
    }
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    return apply_impl(op, kind, in, out, st, scr);  // work fields set: apply_impl allocates nothing
}

static double apply_bytes(bq_op op, int kind, int prec, int ncol, int recon)
{
    const double Vh = op->gauge->g.Vh;
    const double rb = prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2);
    const double sc = prec == PREC_F16 ? 4 : 0;  // per-site scale of an FP16 spinor
    const double spin = 24 * rb + sc;
    const double links = 8 * recon * rb;
    const double clov = 72 * rb;
    switch (kind) {
    case BQ_OP_DEO: case BQ_OP_DOE: case BQ_OP_DEO_DAG: case BQ_OP_DOE_DAG:
        return Vh * (links + ncol * 2 * spin);
    case BQ_OP_K1: case BQ_OP_K1_DAG:
        return Vh * (links + clov + ncol * 2 * spin);
    case BQ_OP_MHAT: case BQ_OP_MHATDAG:  // K1 + K2 (K2 reads v and t, writes out)
        return Vh * (2 * links + 2 * clov + ncol * 5 * spin);
    case BQ_OP_MHATDAG_MHAT:
        return 2 * Vh * (2 * links + 2 * clov + ncol * 5 * spin);
    case BQ_OP_M: case BQ_OP_MDAG:
        return 2 * Vh * (links + clov + ncol * 3 * spin);
    case BQ_OP_MDAGM:
        return 4 * Vh * (links + clov + ncol * 3 * spin);
    case BQ_OP_CLOVER:
        return 2 * Vh * (clov + ncol * 2 * spin);
    case BQ_OP_CLOVER_INV:
        return Vh * (clov + ncol * 2 * spin);
    }
    return 0;
}

int bq_time_apply(bq_op op, int kind, bq_field in, bq_field out, int reps, void* stream, double* ms, double* bytes)
{
    CHK(apply_check(op, kind, in, out));
    if (reps < 1 || !ms) return fail(BQ_ERR_INVALID, "reps must be >= 1 and ms non-NULL");
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    Scratch scr;
    CHK(apply_impl(op, kind, in, out, st, scr));  // warm-up, allocates scratch
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int i = 0; i < reps; i++) CHK(apply_impl(op, kind, in, out, st, scr));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    if (bytes) *bytes = apply_bytes(op, kind, in->prec, in->nrhs, get_tune(ctx, in->prec, in->nrhs).recon);
    return BQ_OK;
}

int bq_time_copy(bq_context ctx, uint64_t bytes, int reps, void* stream, double* ms)
{
    if (!ctx || !ms || reps < 1 || bytes < 16 || bytes % 16) return fail(BQ_ERR_INVALID, "bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    DevBuf a, b;
    CHK(a.alloc(ctx, bytes));
    CHK(b.alloc(ctx, bytes));
    HIPCHK(hipMemsetAsync(a.p, 0, bytes, st));
    HIPCHK(launch_copy16(a.p, b.p, bytes / 16, st));  // warm-up
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int i = 0; i < reps; i++) HIPCHK(launch_copy16(a.p, b.p, bytes / 16, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return BQ_OK;
}

// the checks every solver entry point applies to its parameters
static int check_solve_params(const bq_solve_params& p)
{
    if (!(p.tol > 0) || !std::isfinite(p.tol)) return fail(BQ_ERR_INVALID, "tol must be > 0");
    if (p.inner_prec < BQ_F64 || p.inner_prec > BQ_F16) return fail(BQ_ERR_INVALID, "bad inner precision");
    if (p.system < BQ_SYS_NORMAL || p.system > BQ_SYS_MHAT) return fail(BQ_ERR_INVALID, "bad system");
    if (p.solver < BQ_SOLVER_CG || p.solver > BQ_SOLVER_BLOCK_CG) return fail(BQ_ERR_INVALID, "bad solver");
    if (p.system == BQ_SYS_FULL_NORMAL && (p.inner_prec != BQ_F64 || p.solver != BQ_SOLVER_CG))
        return fail(BQ_ERR_UNSUPPORTED, "the unpreconditioned system is solved by FP64 CG only");
    if (p.solver == BQ_SOLVER_BICGSTAB) {
        if (p.system != BQ_SYS_M && p.system != BQ_SYS_MHAT)
            return fail(BQ_ERR_UNSUPPORTED, "BiCGstab solves M x = b (BQ_SYS_M) or Mhat x = b (BQ_SYS_MHAT)");
        if (p.inner_prec == BQ_F16) return fail(BQ_ERR_UNSUPPORTED, "BiCGstab iterates in FP64 or FP32");
    }
    if (p.solver == BQ_SOLVER_BLOCK_CG && p.inner_prec != BQ_F64)
        return fail(BQ_ERR_UNSUPPORTED, "block CG iterates in FP64");
    if (p.solver == BQ_SOLVER_BLOCK_CG && p.system == BQ_SYS_FULL_NORMAL)
        return fail(BQ_ERR_UNSUPPORTED, "block CG solves the even-odd systems");
    if (p.solver != BQ_SOLVER_CG && p.use_graph) return fail(BQ_ERR_UNSUPPORTED, "graph capture is for CG only");
    if (p.maxiter < 0 || p.chunk < 0 || !(p.delta >= 0) || !(p.delta < 1))
        return fail(BQ_ERR_INVALID, "maxiter and chunk must be >= 0 and delta in [0, 1)");
    return BQ_OK;
}

int bq_solve(bq_op op, bq_field b, bq_field x, const bq_solve_params* params, bq_solve_info* info, void* stream)
{
    if (!op || !b || !x || !params) return fail(BQ_ERR_INVALID, "NULL argument");
    const bq_solve_params& p = *params;
    CHK(check_solve_params(p));
    const int want = (p.system == BQ_SYS_NORMAL || p.system == BQ_SYS_MHAT) ? BQ_ODD : BQ_FULL;
    if (b->subset != want || x->subset != want) return fail(BQ_ERR_INVALID, "b and x must be %s fields", want == BQ_ODD ? "ODD" : "FULL");
    if (b->prec != BQ_F64 || x->prec != BQ_F64) return fail(BQ_ERR_INVALID, "b and x must be FP64 fields");
    if (b->nrhs != x->nrhs) return fail(BQ_ERR_INVALID, "b and x have different nrhs");
    if (b == x) return fail(BQ_ERR_INVALID, "b and x must be different fields");
    if (p.solver == BQ_SOLVER_BLOCK_CG && b->nrhs > kBlockMax)
        return fail(BQ_ERR_UNSUPPORTED, "block CG takes at most %d right-hand sides", kBlockMax);
    for (int k = 0; k < 4; k++)
        if (b->dims[k] != op->gauge->dims[k] || x->dims[k] != op->gauge->dims[k])
            return fail(BQ_ERR_INVALID, "field and gauge lattices differ");
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    CHK(sync_with(ctx, (hipStream_t)stream));
    Vec be, bo, xe, xo;
    if (want == BQ_FULL) {
        be = parity_vec(b, 0);
        bo = parity_vec(b, 1);
        xe = parity_vec(x, 0);
        xo = parity_vec(x, 1);
    } else {
        bo = parity_vec(b, 1);
        xo = parity_vec(x, 1);
    }
    SolveAcct acct;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, ctx->stream));
    int rc;
    if (p.solver == BQ_SOLVER_BICGSTAB)
        rc = bicg_views(op, be, bo, xe, xo, b->nrhs, p, info, ctx->stream, acct);
    else  // CG and block CG share the system preparation, the residuals and the reconstruction
        rc = solve_views(op, be, bo, xe, xo, b->nrhs, p, info, ctx->stream, acct);
    HIPCHK(hipEventRecord(e1, ctx->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->last.bytes = acct.bytes;
    op->last.seconds = ms * 1e-3;
    op->last.launches = acct.launches;
    op->last.chunks = acct.chunks;
    op->last.iterations = acct.iterations;
    return rc;
}

// Block multishift CG: every column of b and every shift in one block Krylov space; per shift
// and column the FP64 residual |b - (Mhat^dag Mhat + sigma) x| is recomputed at the end.
static int ms_block(bq_op op, bq_field b, int nshift, const double* shifts, int base, bq_field* x,
                    const bq_solve_params& prm, bq_solve_info* info, hipStream_t st)
{
    bq_context ctx = op->gauge->ctx;
    const Geom& g = op->gauge->g;
    const int ncol = b->nrhs;
    if (ncol > kBlockMax) return fail(BQ_ERR_UNSUPPORTED, "block CG takes at most %d right-hand sides", kBlockMax);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    SolveAcct acct;
    const Vec bv = parity_vec(b, 1);
    std::vector<Vec> xv(nshift);
    for (int k = 0; k < nshift; k++) xv[k] = parity_vec(x[k], 1);
    BlockOut o;
    CHK(block_engine(op, bv, ncol, nshift, shifts, base, xv.data(), prm, false, st, acct, o));
    // FP64 residuals per shift
    DevBuf dq, sq, dt, stt, dw, sw, part, sum;
    Vec q, t, w;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dq, sq, q));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dt, stt, t));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dw, sw, w));
    const int hw = pad_sites(g.Vh) / kTile;
    const int n = (int)bv.half_sites;
    CHK(part.alloc(ctx, sizeof(double) * (size_t)hw * ncol));
    CHK(sum.alloc(ctx, sizeof(double) * (size_t)ncol));
    double* pr = part.as<double>();
    OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, nullptr, 1, st};
    std::vector<double> b2(ncol), r2((size_t)nshift * ncol);
    HIPCHK(launch_norm2(PREC_F64, bv.all(), n, ncol, pr, hw, st));
    HIPCHK(launch_fin_sum(pr, hw, ncol, sum.as<double>(), st));
    HIPCHK(hipMemcpyAsync(b2.data(), sum.p, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
    for (int k = 0; k < nshift; k++) {
        CHK(op_fwd(c64, 0, xv[k], q, t, nullptr, hw));
        CHK(op_dag_r(c64, 0, q, t, bv, w, nullptr, nullptr, hw));
        HIPCHK(launch_axpy_norm(xv[k].all(), w.all(), -shifts[k], n, ncol, pr, hw, st));
        HIPCHK(launch_fin_sum(pr, hw, ncol, sum.as<double>(), st));
        HIPCHK(hipMemcpyAsync(r2.data() + (size_t)k * ncol, sum.p, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    acct.bytes += nshift * (iter_shared_bytes(op, PREC_F64) + ncol * g.Vh * sp_bytes(PREC_F64) * 13);
    acct.launches += 8L * nshift;
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->last.bytes = acct.bytes;
    op->last.seconds = ms * 1e-3;
    op->last.launches = acct.launches;
    op->last.chunks = acct.chunks;
    op->last.iterations = acct.iterations;
    int rc = BQ_OK;
    for (int k = 0; k < nshift; k++)
        for (int cc = 0; cc < ncol; cc++) {
            const size_t e = (size_t)k * ncol + cc;
            const double tr = b2[cc] > 0 ? std::sqrt(r2[e] / b2[cc]) : 0.0;
            int cst = BQ_OK;
            if (o.failed[cc] || !std::isfinite(tr)) cst = BQ_ERR_NONFINITE;
            else if (!o.conv[e]) cst = BQ_ERR_NOT_CONVERGED;
            if (info) {
                bq_solve_info& in = info[e];
                in.iters = o.iters[e];
                in.reliable_updates = 0;
                in.true_rel_resid = tr;
                in.full_rel_resid = tr;
                in.converged = cst == BQ_OK;
                in.status = cst;
            }
            if (cst == BQ_ERR_NONFINITE) rc = cst;
            else if (cst != BQ_OK && rc == BQ_OK) rc = cst;
        }
    if (rc == BQ_ERR_NOT_CONVERGED) return fail(rc, "some shift did not converge within maxiter");
    if (rc == BQ_ERR_NONFINITE) return fail(rc, "non-finite value in the source or during the solve");
    return BQ_OK;
}

// Multishift CG (the solver list's "multishift cg", the RHMC solver): all shifts share the Krylov
// space of the base system A + sigma_b, sigma_b the smallest shift; shifted residuals stay
// collinear with the base residual, r_k = zeta_k r, and each shift's solution and direction are
// updated with its own alpha_k, beta_k from the zeta recurrence (Jegerlehner's shifted CG).
// One M-hat-dagger-M-hat application per iteration serves every shift and every column.
int bq_solve_multishift(bq_op op, bq_field b, int nshift, const double* shifts, bq_field* x,
                        const bq_solve_params* params, bq_solve_info* info, void* stream)
{
    if (!op || !b || !shifts || !x || !params) return fail(BQ_ERR_INVALID, "NULL argument");
    const bq_solve_params& prm = *params;
    CHK(check_solve_params(prm));
    if (prm.system != BQ_SYS_NORMAL) return fail(BQ_ERR_INVALID, "multishift CG solves Mhat^dag Mhat + sigma (BQ_SYS_NORMAL)");
    if (prm.inner_prec != BQ_F64) return fail(BQ_ERR_UNSUPPORTED, "multishift CG runs in FP64");
    if (nshift < 1 || nshift > kMaxShifts) return fail(BQ_ERR_INVALID, "nshift must be in 1..%d", kMaxShifts);
    int base = 0;
    for (int k = 0; k < nshift; k++) {
        if (!std::isfinite(shifts[k]) || shifts[k] < 0) return fail(BQ_ERR_INVALID, "shifts must be finite and >= 0");
        if (shifts[k] < shifts[base]) base = k;
    }
    if (b->subset != BQ_ODD || b->prec != BQ_F64) return fail(BQ_ERR_INVALID, "b must be an ODD FP64 field");
    for (int k = 0; k < nshift; k++) {
        if (!x[k] || x[k]->subset != BQ_ODD || x[k]->prec != BQ_F64 || x[k]->nrhs != b->nrhs || x[k] == b)
            return fail(BQ_ERR_INVALID, "x[%d] must be an ODD FP64 field with b's nrhs, other than b", k);
        for (int q = 0; q < k; q++)
            if (x[q] == x[k]) return fail(BQ_ERR_INVALID, "x[%d] and x[%d] are the same field", q, k);
        for (int m = 0; m < 4; m++)
            if (x[k]->dims[m] != op->gauge->dims[m]) return fail(BQ_ERR_INVALID, "field and gauge lattices differ");
    }
    for (int m = 0; m < 4; m++)
        if (b->dims[m] != op->gauge->dims[m]) return fail(BQ_ERR_INVALID, "field and gauge lattices differ");
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    CHK(sync_with(ctx, (hipStream_t)stream));
    hipStream_t st = ctx->stream;
    if (prm.solver == BQ_SOLVER_BLOCK_CG) return ms_block(op, b, nshift, shifts, base, x, prm, info, st);
    const Geom& g = op->gauge->g;
    const int ncol = b->nrhs;
    const double sb = shifts[base], kap = op->kappa;

    // workspace: r, p, w, q (odd), t (even), a direction per shift other than the base
    DevBuf dr, sr, dp, spp, dw, sw, dq, sq, dt, stt;
    Vec r, p, w, q, t;
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dr, sr, r));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dp, spp, p));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dw, sw, w));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dq, sq, q));
    CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, dt, stt, t));
    std::vector<std::unique_ptr<DevBuf>> pkbuf;
    MsFields f{};
    f.r = r.all();
    f.w = w.all();
    f.p = p.all();
    for (int k = 0; k < nshift; k++) {
        f.x[k] = parity_vec(x[k], 1).all();
        if (k == base) {
            f.pk[k] = p.all();
            continue;
        }
        pkbuf.emplace_back(new DevBuf);
        DevBuf dummy;
        Vec v;
        CHK(alloc_vec(ctx, g, PREC_F64, 1, ncol, *pkbuf.back(), dummy, v));
        f.pk[k] = v.all();
    }
    const int hw = pad_sites(g.Vh) / kTile;
    const int n = (int)r.half_sites;
    DevBuf part, scal, ints;
    CHK(part.alloc(ctx, sizeof(double) * (size_t)hw * ncol * 3));
    double* pq = part.as<double>();
    double* pr = pq + (size_t)hw * ncol;
    double* pp = pr + (size_t)hw * ncol;
    const size_t ns = (size_t)ncol * nshift;
    CHK(scal.alloc(ctx, sizeof(double) * (8 * (size_t)ncol + 5 * ns)));
    CHK(ints.alloc(ctx, sizeof(int) * (2 * (size_t)ncol + 2 * ns)));
    MsState S{};
    {
        double* d = scal.as<double>();
        S.rho = d; S.alpha = d + ncol; S.alpha_prev = d + 2 * ncol; S.beta = d + 3 * ncol;
        S.beta_prev = d + 4 * ncol; S.stop2 = d + 5 * ncol;
        double* e = d + 8 * (size_t)ncol;
        S.zeta = e; S.zeta_prev = e + ns; S.zeta_new = e + 2 * ns; S.ak = e + 3 * ns; S.bk = e + 4 * ns;
        int* i = ints.as<int>();
        S.status = i; S.iters = i + ncol; S.act = i + 2 * ncol; S.kiters = i + 2 * ncol + ns;
        S.nshift = nshift;
        S.base = base;
        for (int k = 0; k < nshift; k++) S.shift[k] = shifts[k] - sb;
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    const FieldArg bo = parity_vec(b, 1).all();
    SolveAcct acct;
    HIPCHK(launch_convert(PREC_F64, bo, PREC_F64, f.r, n, ncol, nullptr, 0, st));
    HIPCHK(launch_convert(PREC_F64, bo, PREC_F64, f.p, n, ncol, nullptr, 0, st));
    for (int k = 0; k < nshift; k++) {
        HIPCHK(launch_zero(PREC_F64, f.x[k], n, ncol, nullptr, 0, st));
        if (k != base) HIPCHK(launch_convert(PREC_F64, bo, PREC_F64, f.pk[k], n, ncol, nullptr, 0, st));
    }
    HIPCHK(launch_norm2(PREC_F64, f.p, n, ncol, pp, hw, st));
    HIPCHK(launch_fin_sum(pp, hw, ncol, S.rho, st));
    HIPCHK(launch_ms_init(S, ncol, prm.tol * prm.tol, st));
    std::vector<double> b2(ncol);
    HIPCHK(hipMemcpyAsync(b2.data(), S.rho, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));

    const int kchunk = prm.chunk > 0 ? prm.chunk : 8;
    const long maxiter = prm.maxiter > 0 ? prm.maxiter : 100000;
    OpCall c{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, S.status, 1 << COL_ACTIVE, st};
    std::vector<int> hs(ncol);
    long done_iters = 0;
    while (true) {
        for (int it = 0; it < kchunk; it++) {
            CHK(k1(c, 0, f.p, t.all()));
            CHK(tv(c, 0, 1, t.all(), f.p, q.all(), -kap * kap, pq, hw, hw));
            HIPCHK(launch_fin_ms_alpha(S, pq, pp, hw, ncol, sb, st));
            CHK(k1(c, 1, q.all(), t.all()));
            CHK(tv(c, 1, 1, t.all(), q.all(), f.w, -kap * kap, nullptr, hw, hw));
            HIPCHK(launch_ms_update1(S, f, sb, n, ncol, pr, hw, st));
            HIPCHK(launch_fin_ms_beta(S, pr, hw, ncol, st));
            HIPCHK(launch_ms_update2(S, f, n, ncol, pp, hw, st));
        }
        done_iters += kchunk;
        acct.chunks++;
        acct.iterations += kchunk;
        acct.launches += 8L * kchunk;
        HIPCHK(hipMemcpyAsync(hs.data(), S.status, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool all = true;
        for (int cc = 0; cc < ncol; cc++)
            if (hs[cc] == COL_ACTIVE) all = false;
        if (all || done_iters >= maxiter) break;
    }
    std::vector<int> kit(ns), act(ns), cit(ncol);
    HIPCHK(hipMemcpyAsync(kit.data(), S.kiters, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(act.data(), S.act, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(cit.data(), S.iters, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
    // true residuals |b - (Mhat^dag Mhat + sigma_k) x_k| in FP64
    std::vector<double> r2(ns);
    OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, ncol), ncol, nullptr, 1, st};
    Vec bv = parity_vec(b, 1);
    for (int k = 0; k < nshift; k++) {
        Vec xk = parity_vec(x[k], 1);
        CHK(op_fwd(c64, 0, xk, q, t, nullptr, hw));
        CHK(op_dag_r(c64, 0, q, t, bv, w, nullptr, nullptr, hw));
        HIPCHK(launch_axpy_norm(xk.all(), f.w, -shifts[k], n, ncol, pr, hw, st));
        HIPCHK(launch_fin_sum(pr, hw, ncol, S.rho, st));
        HIPCHK(hipMemcpyAsync(r2.data() + (size_t)k * ncol, S.rho, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // bytes: per iteration the four stencil launches, per active column their spinors and the base
    // vectors, per active shift its x (rw) and direction (r, and rw unless it is the base)
    {
        const double Vh = g.Vh, s64 = sp_bytes(PREC_F64);
        long long colit = 0, shit = 0, shit_nb = 0;
        for (int cc = 0; cc < ncol; cc++) colit += cit[cc];
        for (int cc = 0; cc < ncol; cc++)
            for (int k = 0; k < nshift; k++) {
                shit += kit[(size_t)cc * nshift + k];
                if (k != base) shit_nb += kit[(size_t)cc * nshift + k];
            }
        int lock = 0;
        for (int cc = 0; cc < ncol; cc++) lock = std::max(lock, cit[cc]);
        acct.bytes += lock * iter_shared_bytes(op, PREC_F64);
        acct.bytes += colit * Vh * s64 * (9 + 4 + 1 + 3);   // stencils, update1 base, update2 base
        acct.bytes += shit * Vh * s64 * 3 + shit_nb * Vh * s64 * 2;
        acct.bytes += nshift * (iter_shared_bytes(op, PREC_F64) + ncol * Vh * s64 * 13);  // true residuals
    }
    op->last.bytes = acct.bytes;
    op->last.seconds = ms * 1e-3;
    op->last.launches = acct.launches + 8L * nshift;
    op->last.chunks = acct.chunks;
    op->last.iterations = acct.iterations;
    int rc = BQ_OK;
    for (int k = 0; k < nshift; k++)
        for (int cc = 0; cc < ncol; cc++) {
            const size_t i = (size_t)cc * nshift + k;
            const double tr = b2[cc] > 0 ? std::sqrt(r2[(size_t)k * ncol + cc] / b2[cc]) : 0.0;
            int cst = BQ_OK;
            if (!std::isfinite(tr) || hs[cc] == COL_FAILED) cst = std::isfinite(tr) ? BQ_ERR_NOT_CONVERGED : BQ_ERR_NONFINITE;
            else if (act[i]) cst = BQ_ERR_NOT_CONVERGED;
            if (info) {
                bq_solve_info& in = info[(size_t)k * ncol + cc];
                in.iters = kit[i];
                in.reliable_updates = 0;
                in.true_rel_resid = tr;
                in.full_rel_resid = tr;
                in.converged = cst == BQ_OK;
                in.status = cst;
            }
            if (cst == BQ_ERR_NONFINITE) rc = cst;
            else if (cst != BQ_OK && rc == BQ_OK) rc = cst;
        }
    if (rc == BQ_ERR_NOT_CONVERGED) return fail(rc, "some shift did not converge within maxiter");
    if (rc == BQ_ERR_NONFINITE) return fail(rc, "non-finite value in the source or during the solve");
    return BQ_OK;
}

int bq_solve_stats_get(bq_op op, bq_solve_stats* out)
{
    if (!op || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    *out = op->last;
    return BQ_OK;
}

int bq_trace(bq_op op, uint64_t seed, int nnoise, int block, const bq_solve_params* params, double* t1, double* t2,
             bq_solve_info* info)
{
    if (!op || !params || !t1 || !t2) return fail(BQ_ERR_INVALID, "NULL argument");
    if (nnoise < 1 || block < 1) return fail(BQ_ERR_INVALID, "nnoise and block must be >= 1");
    bq_solve_params p = *params;
    p.system = BQ_SYS_M;
    CHK(check_solve_params(p));
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const int* d = op->gauge->dims;
    const Geom& g = op->gauge->g;
    bq_field fa = nullptr, fb = nullptr;
    int rc = bq_field_create(ctx, d, BQ_FULL, BQ_F64, std::min(block, nnoise), &fa);
    if (rc == BQ_OK) rc = bq_field_create(ctx, d, BQ_FULL, BQ_F64, std::min(block, nnoise), &fb);
    FieldPtr ua(fa), ub(fb);
    if (rc != BQ_OK) return rc;
    hipStream_t st = ctx->stream;
    DevBuf part, sums;
    const int nw = (int)(2 * fa->half_sites / kTile);
    CHK(part.alloc(ctx, sizeof(double) * 2 * block * nw));
    CHK(sums.alloc(ctx, sizeof(double) * 2 * block));
    int worst = BQ_OK;
    SolveAcct acct;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int n0 = 0; n0 < nnoise; n0 += block) {
        const int nb = std::min(block, nnoise - n0);
        Vec ae = parity_vec(fa, 0), ao = parity_vec(fa, 1), be_ = parity_vec(fb, 0), bo = parity_vec(fb, 1);
        // eta -> a
        for (int par = 0; par < 2; par++)
            HIPCHK(launch_z2_noise(seed, n0, g, par, parity_vec(fa, par).all(), nb, st));
        // x1 = M^-1 eta -> b
        acct.bytes += 2.0 * nb * 2 * g.Vh * sp_bytes(PREC_F64);  // noise written (both parities)
        int r1 = solve_views(op, ae, ao, be_, bo, nb, p, info ? info + n0 : nullptr, st, acct);
        if (r1 != BQ_OK && r1 != BQ_ERR_NOT_CONVERGED) return r1;
        if (r1 != BQ_OK) worst = r1;
        // t1 = eta^dag x1
        Vec va = field_vec(fa, 0, 2), vb = field_vec(fb, 0, 2);
        HIPCHK(launch_dot(PREC_F64, va.all(), vb.all(), va.sites(), nb, part.as<double>(), nw, st));
        HIPCHK(launch_fin_sum(part.as<double>(), nw, 2 * nb, sums.as<double>(), st));
        HIPCHK(hipMemcpyAsync(t1 + 2 * n0, sums.p, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
        // x2 = M^-1 x1 -> a
        int r2 = solve_views(op, be_, bo, ae, ao, nb, p, info ? info + nnoise + n0 : nullptr, st, acct);
        if (r2 != BQ_OK && r2 != BQ_ERR_NOT_CONVERGED) return r2;
        if (r2 != BQ_OK) worst = r2;
        // eta again -> b ; t2 = eta^dag x2
        for (int par = 0; par < 2; par++)
            HIPCHK(launch_z2_noise(seed, n0, g, par, parity_vec(fb, par).all(), nb, st));
        HIPCHK(launch_dot(PREC_F64, vb.all(), va.all(), va.sites(), nb, part.as<double>(), nw, st));
        HIPCHK(launch_fin_sum(part.as<double>(), nw, 2 * nb, sums.as<double>(), st));
        HIPCHK(hipMemcpyAsync(t2 + 2 * n0, sums.p, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        acct.bytes += 2.0 * nb * 2 * 2 * g.Vh * sp_bytes(PREC_F64) + 2.0 * nb * 2 * g.Vh * sp_bytes(PREC_F64);
        acct.launches += 8;
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->last.bytes = acct.bytes;
    op->last.seconds = ms * 1e-3;
    op->last.launches = acct.launches;
    op->last.chunks = acct.chunks;
    op->last.iterations = acct.iterations;
    if (worst != BQ_OK) return fail(worst, "some trace solve did not converge");
    return BQ_OK;
}

// Per noise eta (complex Z2, as bq_trace) and x1 = M^-1 eta, x2 = M^-1 x1, the terms whose noise
// averages are the traces of the Measurements section and the abstract's reweighting traces:
//   eta^dag x1, eta^dag x2, eta^dag gamma_5 x1, |x1|^2,
//   eta^dag (dM/dkappa) x1 = eta^dag (c_SW S x1 - D x1),  eta^dag (dM/dc_SW) x1 = kappa eta^dag S x1,
//   eta^dag (dM/dmu) x1 = -kappa eta^dag (dD/dmu) x1,
// with S = (T - 1)/(kappa c_SW) the gauge field's clover term without its coefficient and dD/dmu
// the time hops with e^{+mu} (forward) and -e^{-mu} (backward).
int bq_trace_estimators(bq_op op, uint64_t seed, int nnoise, int block, const bq_solve_params* params, double* est,
                        bq_solve_info* info)
{
    if (!op || !params || !est) return fail(BQ_ERR_INVALID, "NULL argument");
    if (nnoise < 1 || block < 1) return fail(BQ_ERR_INVALID, "nnoise and block must be >= 1");
    bq_solve_params p = *params;
    p.system = BQ_SYS_M;
    CHK(check_solve_params(p));
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const int* d = op->gauge->dims;
    const Geom& g = op->gauge->g;
    const int nbmax = std::min(block, nnoise);
    bq_field fa = nullptr, fb = nullptr, fc = nullptr;
    int rc = bq_field_create(ctx, d, BQ_FULL, BQ_F64, nbmax, &fa);
    if (rc == BQ_OK) rc = bq_field_create(ctx, d, BQ_FULL, BQ_F64, nbmax, &fb);
    if (rc == BQ_OK) rc = bq_field_create(ctx, d, BQ_FULL, BQ_F64, nbmax, &fc);
    FieldPtr ua(fa), ub(fb), uc(fc);
    if (rc != BQ_OK) return rc;
    hipStream_t st = ctx->stream;
    DevBuf part, sums;
    const int nw = (int)(2 * fa->half_sites / kTile);
    CHK(part.alloc(ctx, sizeof(double) * 2 * nbmax * nw));
    CHK(sums.alloc(ctx, sizeof(double) * 2 * nbmax * BQ_TR_COUNT));
    double* dsum = sums.as<double>();
    int worst = BQ_OK;
    SolveAcct acct;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    const double kap = op->kappa, csw = op->csw, mu = op->mu;
    const double s64 = sp_bytes(PREC_F64);
    for (int n0 = 0; n0 < nnoise; n0 += block) {
        const int nb = std::min(block, nnoise - n0);
        OpCall c64{op, PREC_F64, get_tune(ctx, PREC_F64, nb), nb, nullptr, 1, st};
        Vec a[2] = {parity_vec(fa, 0), parity_vec(fa, 1)}, b[2] = {parity_vec(fb, 0), parity_vec(fb, 1)},
            cc[2] = {parity_vec(fc, 0), parity_vec(fc, 1)};
        Vec va = field_vec(fa, 0, 2), vb = field_vec(fb, 0, 2), vc = field_vec(fc, 0, 2);
        const int n = va.sites();
        // <x, y> (or <x, gamma_5 y>) of the block's columns into dsum[term][col][re, im]
        auto dot = [&](const Vec& x, const Vec& y, int term, int g5) -> int {
            HIPCHK(launch_dot(PREC_F64, x.all(), y.all(), n, nb, part.as<double>(), nw, st, g5));
            HIPCHK(launch_fin_sum(part.as<double>(), nw, 2 * nb, dsum + (size_t)term * 2 * nbmax, st));
            acct.bytes += 2.0 * nb * n * s64;
            acct.launches += 2;
            return BQ_OK;
        };
        for (int par = 0; par < 2; par++) HIPCHK(launch_z2_noise(seed, n0, g, par, a[par].all(), nb, st));
        acct.bytes += (double)nb * n * s64;
        // x1 = M^-1 eta
        int r1 = solve_views(op, a[0], a[1], b[0], b[1], nb, p, info ? info + n0 : nullptr, st, acct);
        if (r1 != BQ_OK && r1 != BQ_ERR_NOT_CONVERGED) return r1;
        if (r1 != BQ_OK) worst = r1;
        CHK(dot(va, vb, BQ_TR_MINV, 0));
        CHK(dot(va, vb, BQ_TR_G5_MINV, 1));
        CHK(dot(vb, vb, BQ_TR_MDAGM_INV, 0));
        // S x1; the c_SW derivative is kappa <eta, S x1>
        for (int par = 0; par < 2; par++)
            HIPCHK(launch_clover_apply(PREC_F64, g, op->gauge->B[par].p, b[par].all(), cc[par].all(), nb, st));
        CHK(dot(va, vc, BQ_TR_DM_DCSW, 0));
        // (dM/dkappa) x1 = c_SW S x1 - D x1, in place
        for (int par = 0; par < 2; par++)
            CHK(hopv(c64, 0, par, b[1 - par].all(), cc[par].all(), cc[par].all(), csw, -1.0));
        CHK(dot(va, vc, BQ_TR_DM_DKAPPA, 0));
        // (dD/dmu) x1 = D'(forward e^{+mu}, backward -e^{-mu}) x1 - D'(no time hops) x1; the mu
        // derivative is -kappa <eta, (dD/dmu) x1>
        for (int par = 0; par < 2; par++) CHK(hop_coef(c64, par, b[1 - par].all(), cc[par].all(), FieldArg(), 0.0, 1.0, 0.0, 0.0));
        for (int par = 0; par < 2; par++)
            CHK(hop_coef(c64, par, b[1 - par].all(), cc[par].all(), cc[par].all(), -1.0, 1.0, std::exp(mu), -std::exp(-mu)));
        CHK(dot(va, vc, BQ_TR_DM_DMU, 0));
        {
            const double sh = stencil_shared(op, PREC_F64), C64 = (double)g.Vh * 72 * 8.0;
            acct.bytes += 2 * C64 + nb * n * 2.0 * s64;                    // S x1
            acct.bytes += 2 * (sh - C64) + nb * n * 3.0 * s64;            // c_SW S x1 - D x1
            acct.bytes += 4 * (sh - C64) + nb * n * 5.0 * s64;            // dD/dmu x1
            acct.launches += 6;
        }
        // x2 = M^-1 x1
        int r2 = solve_views(op, b[0], b[1], cc[0], cc[1], nb, p, info ? info + nnoise + n0 : nullptr, st, acct);
        if (r2 != BQ_OK && r2 != BQ_ERR_NOT_CONVERGED) return r2;
        if (r2 != BQ_OK) worst = r2;
        CHK(dot(va, vc, BQ_TR_MINV2, 0));
        std::vector<double> h((size_t)2 * nbmax * BQ_TR_COUNT);
        HIPCHK(hipMemcpyAsync(h.data(), dsum, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const double scale[BQ_TR_COUNT] = {1, 1, 1, 1, 1, kap, -kap};
        for (int c = 0; c < nb; c++)
            for (int t = 0; t < BQ_TR_COUNT; t++) {
                const double* v = h.data() + ((size_t)t * nbmax + c) * 2;
                est[((size_t)(n0 + c) * BQ_TR_COUNT + t) * 2 + 0] = scale[t] * v[0];
                est[((size_t)(n0 + c) * BQ_TR_COUNT + t) * 2 + 1] = scale[t] * v[1];
            }
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->last.bytes = acct.bytes;
    op->last.seconds = ms * 1e-3;
    op->last.launches = acct.launches;
    op->last.chunks = acct.chunks;
    op->last.iterations = acct.iterations;
    if (worst != BQ_OK) return fail(worst, "some trace solve did not converge");
    return BQ_OK;
}

int bq_tune_get(bq_context ctx, int prec, int nrhs, int* recon, int* R, int* bs, int* march, int* lds, int* order)
{
    if (!ctx || !recon || !R || !bs || !march || !lds || !order) return fail(BQ_ERR_INVALID, "NULL argument");
    Tune t = get_tune(ctx, prec, nrhs);
    *recon = t.recon;
    *R = t.R;
    *bs = t.bs;
    *march = t.march;
    *lds = t.lds;
    *order = t.order;
    return BQ_OK;
}

int bq_tune_set(bq_context ctx, int prec, int nrhs, int recon, int R, int bs, int march, int lds, int order)
{
    if (!ctx) return fail(BQ_ERR_INVALID, "NULL argument");
    const int rprec = prec == PREC_F64 ? PREC_F64 : PREC_F32;
    if (!hop_variant_exists(prec, rprec, recon, R, EPI_TV) || R > nrhs)
        return fail(BQ_ERR_INVALID, "no kernel variant for prec %d recon %d R %d (nrhs %d)", prec, recon, R, nrhs);
    if (bs != 64 && bs != 128 && bs != 256 && bs != 512 && !(lds && bs % 64 == 0 && bs <= 1024))
        return fail(BQ_ERR_INVALID, "bs must be 64, 128, 256 or 512 (with lds: a multiple of 64 up to 1024)");
    if (march < 0) return fail(BQ_ERR_INVALID, "march must be >= 0");
    if (lds < 0 || lds > 2) return fail(BQ_ERR_INVALID, "lds must be 0, 1 or 2");
    if (lds == 2 && R != 1) return fail(BQ_ERR_INVALID, "lds 2 (lane exchange) takes one column per thread");
    if (order < 0 || order > 2) return fail(BQ_ERR_INVALID, "order must be 0, 1 or 2");
    ctx->tune[{prec, nrhs}] = Tune{recon, R, bs, march, lds, order};
    return BQ_OK;
}

int bq_autotune(bq_op op, int prec, int nrhs)
{
    if (!op) return fail(BQ_ERR_INVALID, "NULL argument");
    if (prec < BQ_F64 || prec > BQ_F16 || nrhs < 1) return fail(BQ_ERR_INVALID, "bad precision or nrhs");
    bq_context ctx = op->gauge->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    bq_field fi = nullptr, fo = nullptr;
    CHK(bq_field_create(ctx, op->gauge->dims, BQ_ODD, prec, nrhs, &fi));
    FieldPtr ui(fi);
    CHK(bq_field_create(ctx, op->gauge->dims, BQ_EVEN, prec, nrhs, &fo));
    FieldPtr uo(fo);
    const int rprec = prec == PREC_F64 ? PREC_F64 : PREC_F32;
    const auto had = ctx->tune.find({prec, nrhs});
    const bool had_entry = had != ctx->tune.end();
    const Tune saved = had_entry ? had->second : get_tune(ctx, prec, nrhs);
    auto time_of = [&](const Tune& t, int reps) {
        ctx->tune[{prec, nrhs}] = t;
        double ms = 0;
        return bq_time_apply(op, BQ_OP_K1, fi, fo, reps, nullptr, &ms, nullptr) == BQ_OK ? ms : 1e300;
    };
    // pass 1: every compiled configuration, a few launches each
    std::vector<std::pair<double, Tune>> cand;
    // t-marching segments the lattice allows (whole tiles per (x,y) plane, segment | L_t)
    const Geom& g = op->gauge->g;
    std::vector<int> marches{0};
    if (g.blocked)
        for (int m : {4, 8, 16, 32})
            if (g.L[3] % m == 0) marches.push_back(m);
    for (int march : marches)
        for (int recon : {12, 18})
            for (int R = 1; R <= std::min(nrhs, 4); R++)
                for (int bs : {64, 128, 256, 512}) {
                    if (!hop_variant_exists(prec, rprec, recon, R, EPI_TINV)) continue;
                    if (recon == 12 && !op->gauge->get(prec, 12)) continue;  // not an SU(3) field
                    const Tune t{recon, R, bs, march, 0};
                    const double ms = time_of(t, 5);
                    if (ms < 1e300) cand.push_back({ms, t});
                }
    // tile-shared kernel: one tile per workgroup (no marching), several column groups per tile
    // (R < nrhs), at most 2 columns per thread, bs / 64 waves per workgroup at most; mode 2 (lane
    // exchange of x and y neighbours) with one column per thread and a whole tile's columns
    for (int recon : {12, 18})
        for (int R = 1; R <= std::min(nrhs - 1, 2); R++)
            for (int waves : {4, 6, 8, 12, 16})
                for (int mode : {1, 2}) {
                    if (!hop_variant_exists(prec, rprec, recon, R, EPI_TINV)) continue;
                    if (recon == 12 && !op->gauge->get(prec, 12)) continue;
                    const int G = (nrhs + R - 1) / R;
                    if (waves > G && waves != 4) continue;  // bs / 64 is only a bound on the waves
                    if (mode == 2 && (R != 1 || waves < std::min(G, 16))) continue;
                    if (prec == PREC_F64 && R > 1) continue;  // spills under the 768-thread bound of FP64
                    const Tune t{recon, R, 64 * waves, 0, mode};
                    const double ms = time_of(t, 5);
                    if (ms < 1e300) cand.push_back({ms, t});
                }
    if (cand.empty()) {
        if (had_entry) ctx->tune[{prec, nrhs}] = saved; else ctx->tune.erase({prec, nrhs});
        return fail(BQ_ERR_DEVICE, "no kernel configuration could be timed");
    }
    // pass 2: the configurations within 10% of the fastest, timed again over more launches; of those
    // within 2% of the new fastest the first in candidate order wins (plain and marching kernels by
    // (march, recon, R, bs), then the tile-shared ones), so near-ties resolve the same way from run to run
    double best = 1e300;
    for (auto& c : cand) best = std::min(best, c.first);
    std::vector<std::pair<double, Tune>> fin;
    for (auto& c : cand)
        if (c.first <= 1.10 * best) fin.push_back({time_of(c.second, 20), c.second});
    double best2 = 1e300;
    for (auto& c : fin) best2 = std::min(best2, c.first);
    Tune bt = fin.front().second;
    for (auto& c : fin)
        if (c.first <= 1.02 * best2) {
            bt = c.second;
            break;
        }
    // pass 3: the winner in the other traversals (z slabs per XCD; and those with the column-group
    // chunks one after another per XCD), kept if 2% faster
    if (bt.march == 0) {
        double tb = time_of(bt, 20);
        const Tune base = bt;
        for (int order : {1, 2}) {
            if (order == 1 && !g.blocked) continue;
            Tune ot = base;
            ot.order = order;
            const double t = time_of(ot, 20);
            if (t < 0.98 * tb) {
                bt = ot;
                tb = t;
            }
        }
    }
    ctx->tune[{prec, nrhs}] = bt;
    return BQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// continuous-batching server
//
// One session per (gauge field, mu, inner precision): a multi-column CG workspace of `cap`
// column slots on its own stream.  Sessions advance independently, one chunk of CG
// iterations plus a reliable-update pass at a time, each chunk ending in an event.  A step
//   1. collects every session whose chunk has finished (event query, no wait) and retires
//      the requests whose columns are done: reconstruction of the even sites, FP64 residual
//      check, copy-out, slots and operator freed;
//   2. admits queued requests into the idle sessions when their columns fit in free slots
//      and their operator fits in the HBM budget: the operator (clover for the request's
//      kappa) is built from the gauge field's kappa-independent B, the source is copied
//      into the slots and prepared (bhat, b' = Mhat^dag bhat) on the device for the new
//      columns only;
//   3. launches the next chunk on every idle session with work.
// If no chunk had finished, the step waits until one does and repeats 1-3 once, so a step
// is one unit of progress.  A small lattice's session runs many chunks while a large
// lattice's session runs one, instead of every session moving in lockstep with the slowest.
// Columns of one batch have their own kappa and clover (per-column stencil launches) and
// share the links.  A column's arithmetic does not depend on the other columns, and it
// enters at a chunk boundary, so its result is the same alone and in the mix.
// ---------------------------------------------------------------------------

static const int COL_NEW = 5;     // admitted this step, source being prepared
static const int COL_RETIRE = 6;  // leaving this step
enum { REQ_QUEUED = 0, REQ_RUNNING = 1, REQ_DONE = 2 };

struct Session;

struct Request {
    uint64_t ticket = 0;
    bq_gauge g = nullptr;
    double kappa = 0, csw = 0, mu = 0, tol = 0;
    int nrhs = 0, prec = 0, maxiter = 0;
    const double* b = nullptr;  // canonical host sources (owned by the caller until retirement)
    double* x_host = nullptr;
    bq_op op = nullptr;
    Session* sess = nullptr;
    std::vector<int> slots;
    int state = REQ_QUEUED;
    int rc = BQ_OK;
    int waited = 0;  // steps spent blocked at the head of its session's queue
    std::vector<bq_solve_info> info;
};

struct Session {
    bq_gauge g = nullptr;
    double mu = 0;
    int prec = 0, cap = 0;
    hipStream_t st = nullptr;
    bq_op_s stub;  // gauge and mu for the launch helpers (no clover of its own)
    Workspace w;
    DevBuf dbf, sbf, dxf, sxf, stage, dflags;
    Vec bfull, xfull;
    ColTable ct{};
    std::vector<Request*> slot;
    int* hflags = nullptr;     // pinned: selection flags (cap ints) then per-column tol^2 (cap doubles)
    double* htol2 = nullptr;
    int used = 0;
    hipEvent_t ev = nullptr;  // recorded after each chunk and its status copy-back
    bool busy = false;        // a chunk is in flight
    // Operators of retired requests, kept with their clover arrays: a new request refills one for
    // its kappa and c_SW.  Freeing device memory waits for the whole device, which would stall
    // every other session at each retirement.
    std::vector<bq_op> spare;
    DevBuf flag;  // positive-definiteness flag of the clover builds on this session's stream
    ~Session()
    {
        if (st) (void)hipStreamSynchronize(st);
        for (bq_op o : spare) (void)bq_op_free(o);
        if (ev) (void)hipEventDestroy(ev);
        if (hflags) (void)hipHostFree(hflags);
        if (st) (void)hipStreamDestroy(st);
        if (g) g->nsess--;
    }
};

struct bq_server_s {
    bq_context ctx = nullptr;
    int cap = 16, chunk = 16;
    int backfill = 8;  // steps a blocked request may be passed by narrower ones of its session
    int per_key = 1;   // sessions per (gauge field, mu, inner precision)
    std::vector<std::unique_ptr<Session>> sessions;
    std::vector<Request*> queue;  // FIFO
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next = 1;
};

static FieldArg col_arg(const Vec& v, int half, int col)
{
    FieldArg a = v.half(half);
    a.d = (char*)a.d + (size_t)col * v.cstride * unit_bytes(v.prec);
    if (a.s) a.s += (size_t)col * v.sstride;
    return a;
}

// a new, empty session of key (g, mu, prec)
static int session_new(bq_server S, bq_gauge g, double mu, int prec, Session** out)
{
    auto s = std::make_unique<Session>();
    s->g = g;
    g->nsess++;  // released by the session's destructor
    s->mu = mu;
    s->prec = prec;
    s->cap = S->cap;
    s->stub.gauge = g;
    s->stub.mu = mu;
    bq_context ctx = S->ctx;
    CHK(ws_init(ctx, g->g, s->cap, prec, 0, &s->w));
    s->w.ct = &s->ct;
    CHK(alloc_vec(ctx, g->g, PREC_F64, 2, s->cap, s->dbf, s->sbf, s->bfull));
    CHK(alloc_vec(ctx, g->g, PREC_F64, 2, s->cap, s->dxf, s->sxf, s->xfull));
    CHK(s->dflags.alloc(ctx, sizeof(int) * s->cap + sizeof(double) * s->cap));
    CHK(s->flag.alloc(ctx, sizeof(int)));
    HIPCHK(hipHostMalloc((void**)&s->hflags, sizeof(int) * s->cap + sizeof(double) * s->cap));
    s->htol2 = (double*)(s->hflags + s->cap);
    HIPCHK(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming));
    s->slot.assign(s->cap, nullptr);
    // every slot starts empty: status DONE is inactive for every kernel
    std::vector<int> st(s->cap, COL_DONE);
    HIPCHK(hipMemcpy(s->w.cs.status, st.data(), sizeof(int) * s->cap, hipMemcpyHostToDevice));
    *out = s.get();
    S->sessions.push_back(std::move(s));
    return BQ_OK;
}

// The session request q goes to: the fullest idle session of its key with room for its columns
// (packing narrow requests leaves the key's other sessions free for wide ones), else a new
// session while the key has fewer than S->per_key.  Otherwise *out = nullptr, *all_busy tells
// whether every session of the key has a chunk in flight.  *first: the key's first session,
// which stands for the key in the admission order (nullptr only if none exists yet).
static int session_for(bq_server S, const Request* q, Session** out, Session** first, bool* all_busy)
{
    *out = *first = nullptr;
    *all_busy = true;
    int count = 0;
    for (auto& sp : S->sessions) {
        Session* s = sp.get();
        if (s->g != q->g || s->mu != q->mu || s->prec != q->prec) continue;
        if (!*first) *first = s;
        count++;
        if (s->busy) continue;
        *all_busy = false;
        if (s->cap - s->used >= q->nrhs && (!*out || s->used > (*out)->used)) *out = s;
    }
    if (*out || count >= S->per_key) return BQ_OK;
    CHK(session_new(S, q->g, q->mu, q->prec, out));
    if (!*first) *first = *out;
    *all_busy = false;
    return BQ_OK;
}

// device pointers to the selection flags and per-column tol^2 of a session
static int* dsel(Session* s) { return s->dflags.as<int>(); }
static double* dtol2(Session* s) { return (double*)(s->dflags.as<int>() + s->cap); }

static int admit(bq_server S, Request* q, Session* s)
{
    bq_context ctx = S->ctx;
    const Geom& g = s->g->g;
    if (!s->spare.empty()) {
        bq_op o = s->spare.back();
        s->spare.pop_back();
        const int rc = clover_fill(o, q->kappa, q->csw, s->prec, s->flag.as<int>(), s->st);
        if (rc != BQ_OK) {
            s->spare.push_back(o);
            return rc;
        }
        o->mu = q->mu;
        q->op = o;
    } else {
        CHK(op_build(q->g, q->kappa, q->csw, q->mu, s->prec, &q->op, s->flag.as<int>(), s->st));
    }
    const size_t V = 2 * (size_t)g.Vh;
    const size_t bytes = (size_t)q->nrhs * V * 12 * 16;
    if (s->stage.bytes < bytes) CHK(s->stage.alloc(ctx, bytes));
    HIPCHK(hipMemcpyAsync(s->stage.p, q->b, bytes, hipMemcpyDefault, s->st));  // b in host or device memory
    q->slots.clear();
    for (int c = 0, k = 0; c < s->cap && k < q->nrhs; c++)
        if (!s->slot[c]) {
            s->slot[c] = q;
            q->slots.push_back(c);
            const double2* canon = s->stage.as<double2>() + (size_t)k * V * 12;
            for (int p = 0; p < 2; p++)
                HIPCHK(launch_spinor_import(canon, 1, g, p, PREC_F64, col_arg(s->bfull, p, c), s->st));
            for (int pr = 0; pr < 3; pr++) {
                s->ct.T[pr][1][c] = q->op->T[pr][1].p;
                s->ct.T[pr][0][c] = q->op->T[pr][0].p;
                s->ct.Tinv[pr][0][c] = q->op->Tinv[pr][0].p;
            }
            s->ct.kappa[c] = q->kappa;
            s->hflags[c] = 1;
            s->htol2[c] = q->tol * q->tol;
            k++;
        }
    s->used += q->nrhs;
    q->sess = s;
    q->state = REQ_RUNNING;
    return BQ_OK;
}

// prepare the columns flagged in hflags: b' = Mhat^dag (b_o + kappa D_oe T_ee^-1 b_e), CG state
static int prepare_new(Session* s)
{
    const int cap = s->cap;
    Workspace* w = &s->w;
    hipStream_t st = s->st;
    HIPCHK(hipMemcpyAsync(s->dflags.p, s->hflags, sizeof(int) * cap + sizeof(double) * cap, hipMemcpyHostToDevice, st));
    HIPCHK(launch_set_status(w->cs.status, dsel(s), cap, COL_NEW, st));
    const int m = 1 << COL_NEW;
    OpCall c64{&s->stub, PREC_F64, get_tune(s->g->ctx, PREC_F64, cap), cap, w->cs.status, m, st};
    c64.ct = &s->ct;
    const void* tinv[kMaxCols];
    for (int c = 0; c < cap; c++) tinv[c] = s->ct.Tinv[PREC_F64][0][c];
    HIPCHK(launch_clover_apply(PREC_F64, s->g->g, nullptr, s->bfull.half(0), w->t64.all(), cap, st, tinv, w->cs.status, m));
    CHK(hopv(c64, 0, 1, w->t64.all(), w->q64.all(), s->bfull.half(1), 1.0, 0.0, FK_KAPPA));
    CHK(k1(c64, 1, w->q64.all(), w->t64.all()));
    CHK(tv(c64, 1, 1, w->t64.all(), w->q64.all(), w->bp.all(), 0.0, nullptr, 0, 0, FK_MKAPPA2));
    const int n = w->x.sites();
    HIPCHK(launch_zero(PREC_F64, w->x.all(), n, cap, w->cs.status, m, st));
    HIPCHK(launch_convert(PREC_F64, w->bp.all(), PREC_F64, w->r.all(), n, cap, w->cs.status, m, st));
    if (s->prec != PREC_F64) {
        HIPCHK(launch_zero(w->xs.prec, w->xs.all(), n, cap, w->cs.status, m, st));
        HIPCHK(launch_convert(PREC_F64, w->bp.all(), w->rs.prec, w->rs.all(), n, cap, w->cs.status, m, st));
        HIPCHK(launch_convert(w->rs.prec, w->rs.all(), w->ps.prec, w->ps.all(), n, cap, w->cs.status, m, st));
    } else {
        HIPCHK(launch_convert(PREC_F64, w->bp.all(), PREC_F64, w->ps.all(), n, cap, w->cs.status, m, st));
    }
    HIPCHK(launch_norm2(PREC_F64, w->bp.all(), n, cap, w->partial, w->pstride, st));
    HIPCHK(launch_fin_sum(w->partial, w->pstride, cap, w->dtmp, st));
    HIPCHK(launch_cg_init(w->cs, cap, 0.0, st, dsel(s), dtol2(s), w->dtmp));
    return BQ_OK;
}

// retire the requests in `done` (all on session s): fold, residual check, reconstruct, copy out
static int retire(bq_server S, Session* s, std::vector<Request*>& done)
{
    (void)S;
    const int cap = s->cap;
    Workspace* w = &s->w;
    hipStream_t st = s->st;
    for (int c = 0; c < cap; c++) s->hflags[c] = 0;
    for (Request* q : done)
        for (int c : q->slots) s->hflags[c] = 1;
    HIPCHK(hipMemcpyAsync(s->dflags.p, s->hflags, sizeof(int) * cap, hipMemcpyHostToDevice, st));
    const int n = w->x.sites();
    // columns that stopped on maxiter still hold an inner iterate: fold it in (it is 0 for
    // columns that converged, whose last reliable update folded it)
    HIPCHK(launch_set_status(w->cs.status, dsel(s), cap, COL_RETIRE, st));
    const int m = 1 << COL_RETIRE;
    if (s->prec != PREC_F64) HIPCHK(launch_accum(w->xs.prec, w->xs.all(), w->x.all(), n, cap, w->cs.status, m, st));
    CHK(true_residual(&s->stub, w, w->cs.status, m, st));
    HIPCHK(launch_fin_sum(w->partial, w->pstride, cap, w->dtmp, st));
    HIPCHK(launch_norm2(PREC_F64, w->bp.all(), n, cap, w->partial, w->pstride, st));
    HIPCHK(launch_fin_sum(w->partial, w->pstride, cap, w->dtmp + cap, st));
    // x_o into the full solution, x_e = T_ee^-1 (b_e + kappa D_eo x_o)
    HIPCHK(launch_convert(PREC_F64, w->x.all(), PREC_F64, s->xfull.half(1), n, cap, w->cs.status, m, st));
    OpCall c64{&s->stub, PREC_F64, get_tune(s->g->ctx, PREC_F64, cap), cap, w->cs.status, m, st};
    c64.ct = &s->ct;
    CHK(k1(c64, 0, s->xfull.half(1), s->xfull.half(0), s->bfull.half(0), 1.0, 0.0, FK_KAPPA));
    // |b - M x|^2 on the full lattice (t64 and q64 as even / odd scratch) and |b|^2
    const int hw = w->hw;
    CHK(tvr(c64, 0, 0, s->xfull.half(1), s->xfull.half(0), s->bfull.half(0), w->t64.all(), 0.0, nullptr, w->partial, hw,
            2 * hw, FK_MKAPPA));
    CHK(tvr(c64, 0, 1, s->xfull.half(0), s->xfull.half(1), s->bfull.half(1), w->q64.all(), 0.0, nullptr,
            w->partial + hw, hw, 2 * hw, FK_MKAPPA));
    HIPCHK(launch_fin_sum(w->partial, 2 * hw, cap, w->dtmp + 2 * cap, st));
    HIPCHK(launch_norm2(PREC_F64, s->bfull.all(), s->bfull.sites(), cap, w->partial, 2 * hw, st));
    HIPCHK(launch_fin_sum(w->partial, 2 * hw, cap, w->dtmp + 3 * cap, st));
    std::vector<double> h(4 * cap);
    std::vector<int> hi(4 * cap);
    HIPCHK(hipMemcpyAsync(h.data(), w->dtmp, sizeof(double) * 4 * cap, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hi.data(), w->cs.status, sizeof(int) * 4 * cap, hipMemcpyDeviceToHost, st));
    const Geom& g = s->g->g;
    const size_t V = 2 * (size_t)g.Vh;
    for (Request* q : done) {
        const size_t bytes = (size_t)q->nrhs * V * 12 * 16;
        if (s->stage.bytes < bytes) CHK(s->stage.alloc(S->ctx, bytes));
        for (size_t k = 0; k < q->slots.size(); k++)
            for (int p = 0; p < 2; p++)
                HIPCHK(launch_spinor_export(col_arg(s->xfull, p, q->slots[k]), 1, g, p, PREC_F64,
                                            s->stage.as<double2>() + k * V * 12, st));
        HIPCHK(hipMemcpyAsync(q->x_host, s->stage.p, bytes, hipMemcpyDefault, st));  // x in host or device memory
        HIPCHK(hipStreamSynchronize(st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (Request* q : done) {
        q->info.assign(q->nrhs, bq_solve_info{});
        q->rc = BQ_OK;
        for (size_t k = 0; k < q->slots.size(); k++) {
            const int c = q->slots[k];
            const double tr = h[cap + c] > 0 ? std::sqrt(h[c] / h[cap + c]) : 0.0;
            bq_solve_info& in = q->info[k];
            in.iters = hi[cap + c];
            in.reliable_updates = hi[3 * cap + c];
            in.true_rel_resid = tr;
            in.full_rel_resid = h[3 * cap + c] > 0 ? std::sqrt(h[2 * cap + c] / h[3 * cap + c]) : 0.0;
            in.converged = std::isfinite(tr) && tr <= q->tol;
            in.status = !std::isfinite(tr) ? BQ_ERR_NONFINITE : (in.converged ? BQ_OK : BQ_ERR_NOT_CONVERGED);
            if (in.status != BQ_OK && q->rc == BQ_OK) q->rc = in.status;
            s->slot[c] = nullptr;
            for (int pr = 0; pr < 3; pr++) s->ct.T[pr][0][c] = s->ct.T[pr][1][c] = s->ct.Tinv[pr][0][c] = nullptr;
        }
        s->used -= q->nrhs;
        s->spare.push_back(q->op);
        q->op = nullptr;
        q->state = REQ_DONE;
    }
    HIPCHK(launch_set_status(w->cs.status, dsel(s), cap, COL_DONE, st));
    return BQ_OK;
}

extern "C" {

int bq_server_create(bq_context ctx, int slots, int chunk, bq_server* out)
{
    if (!ctx || !out) return fail(BQ_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (slots < 1 || slots > kMaxCols) return fail(BQ_ERR_INVALID, "slots must be in 1..%d", kMaxCols);
    auto S = std::make_unique<bq_server_s>();
    S->ctx = ctx;
    S->cap = slots;
    S->chunk = chunk > 0 ? chunk : 16;
    *out = S.release();
    ctx->nhandles++;
    return BQ_OK;
}

int bq_server_submit(bq_server S, bq_gauge g, double kappa, double csw, double mu, const double* b, double* x,
                     int nrhs, double tol, int inner_prec, int maxiter, uint64_t* ticket)
{
    if (!S || !g || !b || !x || !ticket) return fail(BQ_ERR_INVALID, "NULL argument");
    if (g->ctx != S->ctx) return fail(BQ_ERR_INVALID, "gauge field of another context");
    if (nrhs < 1 || nrhs > S->cap) return fail(BQ_ERR_INVALID, "nrhs must be in 1..%d", S->cap);
    if (!(tol > 0) || !std::isfinite(tol)) return fail(BQ_ERR_INVALID, "tol must be > 0");
    if (inner_prec < BQ_F64 || inner_prec > BQ_F16) return fail(BQ_ERR_INVALID, "bad inner precision");
    if (!std::isfinite(kappa) || !std::isfinite(csw) || !std::isfinite(mu))
        return fail(BQ_ERR_INVALID, "kappa, c_SW and mu must be finite");
    if (!g->get(PREC_F64, 12) || !g->get(inner_prec, 12))
        return fail(BQ_ERR_UNSUPPORTED, "the server needs two-row links: this gauge field is not SU(3) "
                                        "(max deviation %.3g)", g->su3_dev);
    auto q = std::make_unique<Request>();
    q->ticket = S->next++;
    q->g = g;
    q->kappa = kappa;
    q->csw = csw;
    q->mu = mu;
    q->tol = tol;
    q->nrhs = nrhs;
    q->prec = inner_prec;
    q->maxiter = maxiter > 0 ? maxiter : 100000;
    q->b = b;
    q->x_host = x;
    *ticket = q->ticket;
    S->queue.push_back(q.get());
    S->reqs[q->ticket] = std::move(q);
    return BQ_OK;
}

// A request that cannot be admitted for a reason other than memory (its clover is not positive
// definite, a device call failed) is finished at once with that status; the others go on.
static void finish_failed(Request* q, int rc)
{
    q->state = REQ_DONE;
    q->rc = rc;
    bq_solve_info bad{};
    bad.status = rc;
    q->info.assign(q->nrhs, bad);
}

// undo a partial admission: free the request's slots and operator, back to the queue
static void unadmit(Request* q, Session* s)
{
    for (int c : q->slots) {
        s->slot[c] = nullptr;
        s->hflags[c] = 0;
        for (int pr = 0; pr < 3; pr++) s->ct.T[pr][0][c] = s->ct.T[pr][1][c] = s->ct.Tinv[pr][0][c] = nullptr;
    }
    if (q->op) s->spare.push_back(q->op);
    q->op = nullptr;
    q->slots.clear();
    q->sess = nullptr;
    q->state = REQ_QUEUED;
}

// Free the spare operators of every session, when the HBM budget needs their memory; true if
// there were any.  No work in flight reads a spare operator.
static bool trim_spares(bq_server S)
{
    bool any = false;
    for (auto& sp : S->sessions) {
        for (bq_op o : sp->spare) (void)bq_op_free(o);
        any |= !sp->spare.empty();
        sp->spare.clear();
    }
    return any;
}

// the requests of session s whose columns are all done, stopped or out of iterations, from the
// status copied back at the end of its last chunk; they retire and are reported
static int collect(bq_server S, Session* s, const std::function<void(Request*)>& report)
{
    const int* hs = s->w.h_status;
    std::vector<Request*> done;
    for (int c = 0; c < s->cap; c++) {
        Request* q = s->slot[c];
        if (!q || std::find(done.begin(), done.end(), q) != done.end()) continue;
        bool fin = true;
        for (int cc : q->slots) {
            const int stc = hs[cc];
            const bool out_of_iters = hs[s->cap + cc] >= q->maxiter;
            if (!(stc == COL_DONE || stc == COL_FAILED || out_of_iters)) fin = false;
        }
        if (fin) done.push_back(q);
    }
    if (!done.empty()) {
        CHK(retire(S, s, done));
        for (Request* q : done) report(q);
    }
    return BQ_OK;
}

// 1. of the step: sessions whose chunk has finished become idle and retire what it completed.
// With `wait`, first wait (polling the events) until at least one busy session has finished.
static int poll_sessions(bq_server S, bool wait, bool* progressed, const std::function<void(Request*)>& report)
{
    for (;;) {
        for (auto& sp : S->sessions) {
            Session* s = sp.get();
            if (!s->busy) continue;
            const hipError_t e = hipEventQuery(s->ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(BQ_ERR_DEVICE, "server chunk: %s", hipGetErrorString(e));
            s->busy = false;
            *progressed = true;
            CHK(collect(S, s, report));
        }
        if (!wait || *progressed) return BQ_OK;
        bool any = false;
        for (auto& sp : S->sessions) any |= sp->busy;
        if (!any) return BQ_OK;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// 2. of the step: admission in arrival order per idle session.  A request that does not fit waits
// at the head of its session; later, narrower requests may pass it (backfill) until it has waited
// S->backfill steps, after which the session admits nothing else until it fits.  Requests of a
// session with a chunk in flight stay queued without waiting a step.
static int admit_queued(bq_server S, std::set<Request*>& blocked, const std::function<void(Request*)>& report)
{
    std::vector<Session*> fresh;
    std::vector<Request*> keep;
    std::map<Session*, Request*> head;  // first blocked request per key (its first session)
    for (Request* q : S->queue) {
        Session *s = nullptr, *first = nullptr;
        bool all_busy = true;
        int rc = session_for(S, q, &s, &first, &all_busy);
        if (rc == BQ_ERR_OOM && trim_spares(S)) rc = session_for(S, q, &s, &first, &all_busy);
        if (rc == BQ_ERR_OOM) {  // no memory for a new session: wait for an existing one, if any
            rc = BQ_OK;
            s = nullptr;
            if (!first) {
                keep.push_back(q);
                continue;
            }
        }
        if (rc != BQ_OK) {
            finish_failed(q, rc);
            report(q);
            continue;
        }
        if (!s && all_busy) {  // every session of the key has a chunk in flight: no step is waited
            keep.push_back(q);
            continue;
        }
        Request*& h = head[first];
        const bool may_pass = h == nullptr || h->waited < S->backfill;
        if (!s || !may_pass) {
            if (h == nullptr) h = q;
            keep.push_back(q);
            continue;
        }
        if (std::find(fresh.begin(), fresh.end(), s) == fresh.end()) {
            for (int c = 0; c < s->cap; c++) s->hflags[c] = 0;
            fresh.push_back(s);
        }
        rc = admit(S, q, s);
        if (rc == BQ_ERR_OOM) {  // no room for the operator: free the spare ones and try again
            unadmit(q, s);
            if (trim_spares(S)) rc = admit(S, q, s);
        }
        if (rc == BQ_ERR_OOM) {  // no room for the operator now: undo and wait
            unadmit(q, s);
            if (h == nullptr) h = q;
            keep.push_back(q);
            continue;
        }
        if (rc != BQ_OK) {
            unadmit(q, s);
            finish_failed(q, rc);
            report(q);
            continue;
        }
    }
    for (auto& kv : head)
        if (kv.second) blocked.insert(kv.second);
    S->queue = keep;
    for (Session* s : fresh) {
        bool any = false;
        for (int c = 0; c < s->cap; c++) any |= s->hflags[c] != 0;
        if (any) CHK(prepare_new(s));
    }
    return BQ_OK;
}

// 3. of the step: the next chunk on every idle session with work, ending in its event
static int launch_idle(bq_server S)
{
    for (auto& sp : S->sessions) {
        Session* s = sp.get();
        if (s->busy || s->used == 0) continue;
        Workspace* w = &s->w;
        w->cs.delta2 = s->prec == PREC_F64 ? 0.0 : 0.01;  // reliable-update threshold delta = 0.1
        CHK(chunk(&s->stub, w, s->prec, S->chunk, s->st));
        HIPCHK(hipMemcpyAsync(w->h_status, w->cs.status, sizeof(int) * 4 * s->cap, hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipEventRecord(s->ev, s->st));
        s->busy = true;
    }
    return BQ_OK;
}

int bq_server_step(bq_server S, uint64_t* done_tickets, int max_done, int* ndone)
{
    if (!S || !ndone) return fail(BQ_ERR_INVALID, "NULL argument");
    *ndone = 0;
    bq_context ctx = S->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const std::function<void(Request*)> report = [&](Request* q) {
        if (*ndone < max_done && done_tickets) done_tickets[*ndone] = q->ticket;
        (*ndone)++;
    };
    std::set<Request*> blocked;  // heads that could not be admitted: each waits one step
    bool progressed = false;
    for (int pass = 0; pass < 2; pass++) {
        CHK(poll_sessions(S, pass == 1, &progressed, report));
        CHK(admit_queued(S, blocked, report));
        CHK(launch_idle(S));
        bool any = false;
        for (auto& sp : S->sessions) any |= sp->busy;
        if (progressed || !any) break;
    }
    for (Request* q : blocked)
        if (q->state == REQ_QUEUED) q->waited++;
    return BQ_OK;
}

int bq_server_result(bq_server S, uint64_t ticket, bq_solve_info* info)
{
    if (!S) return fail(BQ_ERR_INVALID, "NULL argument");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(BQ_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Request* q = it->second.get();
    if (q->state != REQ_DONE) return BQ_PENDING;
    if (info)
        for (int k = 0; k < q->nrhs; k++) info[k] = q->info[k];
    const int rc = q->rc;
    S->reqs.erase(it);
    return rc;
}

int bq_server_pending(bq_server S, int* queued, int* running)
{
    if (!S || !queued || !running) return fail(BQ_ERR_INVALID, "NULL argument");
    *queued = (int)S->queue.size();
    int r = 0;
    for (auto& kv : S->reqs)
        if (kv.second->state == REQ_RUNNING) r++;
    *running = r;
    return BQ_OK;
}

int bq_server_set_backfill(bq_server S, int steps)
{
    if (!S || steps < 0) return fail(BQ_ERR_INVALID, "NULL server or negative step count");
    S->backfill = steps;
    return BQ_OK;
}

int bq_server_set_sessions(bq_server S, int per_key)
{
    if (!S || per_key < 1 || per_key > 8) return fail(BQ_ERR_INVALID, "NULL server or sessions per key outside 1..8");
    S->per_key = per_key;
    return BQ_OK;
}

int bq_server_release(bq_server S, bq_gauge g)
{
    if (!S || !g) return fail(BQ_ERR_INVALID, "NULL argument");
    for (auto& kv : S->reqs)
        if (kv.second->g == g && kv.second->state != REQ_DONE)
            return fail(BQ_ERR_BUSY, "request %llu on this gauge field is still queued or running",
                        (unsigned long long)kv.first);
    (void)hipSetDevice(S->ctx->device);
    auto& v = S->sessions;
    v.erase(std::remove_if(v.begin(), v.end(), [g](const std::unique_ptr<Session>& s) { return s->g == g; }), v.end());
    return BQ_OK;
}

int bq_server_free(bq_server S)
{
    if (!S) return BQ_OK;
    (void)hipSetDevice(S->ctx->device);
    for (auto& s : S->sessions) (void)hipStreamSynchronize(s->st);
    for (auto& kv : S->reqs)
        if (kv.second->op) bq_op_free(kv.second->op);
    bq_context ctx = S->ctx;
    delete S;
    ctx_release_handle(ctx);
    return BQ_OK;
}

}  // extern "C"
