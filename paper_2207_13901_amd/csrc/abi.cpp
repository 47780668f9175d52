// C ABI of libspleaf: argument checks, schedule resolution, workspace
// carving and kernel dispatch.  Every entry point catches all C++
// exceptions and converts them to status codes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <map>
#include <memory>

#include "internal.hpp"
#include "spleaf.h"
#include "tin.hpp"

struct spl_context {
    int device = 0;
    std::string err;
    void *ws = nullptr;   // context-owned workspace (used when the caller gives none)
    size_t ws_bytes = 0;
    int64_t *flags = nullptr;  // 2 x int64 device scratch for spl_validate
    // pinned host slot for the counts read back to the host (an output's
    // nonzero count, spl_validate's flags): a copy into pinned memory is a
    // plain DMA, where pageable memory goes through the runtime's staging
    // buffer.  Calls on one context are not meant to overlap across host
    // threads (the error string is shared too).
    int64_t *readback = nullptr;  // 2 x int64
    // leaf-kernel timing (spl_timing_enable / spl_timing_read)
    struct Mark {
        hipEvent_t start, stop;
        int op;
    };
    bool timing = false;
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
    // installed schedule selectors (spl_mlp_*), [0] SpMV, [1] SpMM
    struct Selector {
        int K = 0;
        std::vector<spl_schedule> cands;
        int64_t nparams = 0;
        float *params = nullptr;   // device, the network
        float *norm = nullptr;     // device, 7 means + 7 inverse standard deviations
        float *m = nullptr;        // device, Adam moments
        float *v = nullptr;
        float *scratch = nullptr;  // device, 8 features + K predictions
        int step = 0;
    };
    Selector sel[2];
    hipError_t scratch_status = hipSuccess;  // spl::scratch_init on `device`
    // generated leaves of index-notation statements, by statement and formats
    std::map<std::string, std::unique_ptr<spl::tin::Program>> tin_cache;
};

namespace {

using spl::Tiles;

spl_status fail(spl_context *ctx, spl_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

spl_status hip_fail(spl_context *ctx, hipError_t e, const char *where) {
    return fail(ctx, SPL_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define SPL_GUARD_BEGIN try {
#define SPL_GUARD_END                                                         \
    }                                                                         \
    catch (const std::bad_alloc &) {                                          \
        return fail(ctx, SPL_ERR_NOMEM, "host allocation failed");            \
    }                                                                         \
    catch (...) {                                                             \
        return fail(ctx, SPL_ERR_ARG, "unexpected internal exception");       \
    }

constexpr int64_t kIndexMax = 2147483647;  // int32 pos/crd

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

bool valid_dtype(int dt) { return dt == SPL_F64 || dt == SPL_F32 || dt == SPL_BF16; }

// allow_i64: the caller handles int64 positions (SpMV, SpMM, SpTTV, MTTKRP).
spl_status check_sparse(spl_context *ctx, const spl_sparse *B, int order, bool allow_i64 = false) {
    if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
    if (B->pos_type != SPL_I32 && B->pos_type != SPL_I64)
        return fail(ctx, SPL_ERR_FORMAT, "unknown pos_type %d", B->pos_type);
    if (B->pos_type == SPL_I64 && !allow_i64)
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "int64 positions are accepted by SpMV, SpMM, SpTTV and MTTKRP (MERGE "
                    "schedule) only");
    if (B->order != order)
        return fail(ctx, SPL_ERR_FORMAT, "expected an order-%d sparse operand, got order %d", order,
                    B->order);
    if (B->level[0] != SPL_DENSE)
        return fail(ctx, SPL_ERR_FORMAT, "level 0 must be Dense");
    // a 3-tensor's middle level may be Dense: (Dense, Dense, Compressed)
    const bool dmid = order == 3 && B->level[1] == SPL_DENSE;
    for (int l = 1; l < order; ++l)
        if (B->level[l] != SPL_COMPRESSED && !(l == 1 && dmid))
            return fail(ctx, SPL_ERR_FORMAT, order == 3 && l == 1
                                                 ? "level 1 must be Dense or Compressed"
                                                 : "level %d must be Compressed", l);
    if (!valid_dtype(B->vtype)) return fail(ctx, SPL_ERR_DTYPE, "unknown value dtype %d", B->vtype);
    for (int l = 0; l < order; ++l)
        if (B->dims[l] < 0 || B->dims[l] > kIndexMax)
            return fail(ctx, SPL_ERR_SHAPE, "dimension %d = %lld out of range", l,
                        static_cast<long long>(B->dims[l]));
    const int64_t nnz_max = B->pos_type == SPL_I64 ? (int64_t{1} << 62) : kIndexMax;
    if (B->nnz < 0 || B->nnz > nnz_max)
        return fail(ctx, SPL_ERR_SHAPE, "nnz = %lld out of range", static_cast<long long>(B->nnz));
    if (order == 3 && (B->nfibers < 0 || B->nfibers > kIndexMax))
        return fail(ctx, SPL_ERR_SHAPE, "nfibers = %lld out of range",
                    static_cast<long long>(B->nfibers));
    if (dmid && B->nfibers != B->dims[0] * B->dims[1])
        return fail(ctx, SPL_ERR_SHAPE, "a Dense middle level holds dims[0] * dims[1] fibers");
    for (int l = dmid ? 2 : 1; l < order; ++l) {
        if (!B->pos[l]) return fail(ctx, SPL_ERR_ARG, "pos[%d] is NULL", l);
        const int64_t children = (l == order - 1) ? B->nnz : B->nfibers;
        if (children > 0 && !B->crd[l]) return fail(ctx, SPL_ERR_ARG, "crd[%d] is NULL", l);
    }
    if (B->nnz > 0 && !B->vals) return fail(ctx, SPL_ERR_ARG, "vals is NULL");
    return SPL_OK;
}

spl_status check_dense(spl_context *ctx, const spl_dense *d, const char *name, int ndim,
                       int64_t d0, int64_t d1) {
    if (!d) return fail(ctx, SPL_ERR_ARG, "dense operand %s is NULL", name);
    if (d->ndim != ndim)
        return fail(ctx, SPL_ERR_SHAPE, "%s: expected %d dimensions, got %d", name, ndim, d->ndim);
    if (!valid_dtype(d->dtype)) return fail(ctx, SPL_ERR_DTYPE, "%s: unknown dtype", name);
    if (d->dims[0] != d0 || (ndim == 2 && d1 >= 0 && d->dims[1] != d1))
        return fail(ctx, SPL_ERR_SHAPE, "%s: shape mismatch", name);
    if (ndim == 2 && d->ld < d->dims[1])
        return fail(ctx, SPL_ERR_SHAPE, "%s: leading dimension smaller than its columns", name);
    const int64_t elems = ndim == 1 ? d->dims[0] : d->dims[0] * d->dims[1];
    if (elems > 0 && !d->data) return fail(ctx, SPL_ERR_ARG, "%s: data is NULL", name);
    return SPL_OK;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// Resolved schedule of one call.
struct Plan {
    int kind = SPL_MERGE;
    int lanes = 0;
    int64_t tile = 0;
    int items = 0;
    int col_tile = 0;
    int variant = 0;
    int vec = 1;  // SpMM: dense columns per lane
};

int lanes_for_mean(double mean) {
    int L = 1;
    while (L < 64 && L < mean) L <<= 1;
    return L;
}

// Merged items per SpMV leaf chunk: a workgroup's lanes times the items each
// walks.
int64_t spmv_chunk(const Plan &p) { return 256 * p.items; }

spl_status resolve_spmv(spl_context *ctx, const spl_sparse *B, const spl_schedule *s, Plan &p) {
    spl_schedule d{};
    if (!s) s = &d;
    p.kind = s->kind == SPL_SCHED_DEFAULT ? SPL_MERGE : s->kind;
    if (p.kind != SPL_ROW && p.kind != SPL_NNZ && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "unknown schedule kind %d", s->kind);
    const int64_t n = B->dims[0];
    p.lanes = s->lanes_per_row ? s->lanes_per_row
                               : lanes_for_mean(n ? static_cast<double>(B->nnz) / n : 1.0);
    if (!pow2_in(p.lanes, 1, 64)) return fail(ctx, SPL_ERR_ARG, "lanes_per_row must be 1..64, power of 2");
    p.items = s->items_per_lane ? s->items_per_lane : 8;
    if (p.items != 4 && p.items != 8) return fail(ctx, SPL_ERR_ARG, "SpMV items_per_lane must be 4 or 8");
    if (s->variant < 0 || s->variant > 2)
        return fail(ctx, SPL_ERR_ARG,
                    "SpMV variant must be 0 (row-end flags), 1 (row-end search) or 2 (whole rows "
                    "per lane)");
    if (s->variant != 0 && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "SpMV variants 1 and 2 need the MERGE schedule");
    p.variant = s->variant;
    p.tile = s->tile ? s->tile : (p.kind == SPL_ROW ? 256 / p.lanes : spmv_chunk(p));
    if (p.tile < 1) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    return SPL_OK;
}

spl_status resolve_spmm(spl_context *ctx, const spl_sparse *B, int64_t N, const spl_schedule *s,
                        Plan &p) {
    spl_schedule d{};
    if (!s) s = &d;
    p.kind = s->kind == SPL_SCHED_DEFAULT ? SPL_MERGE : s->kind;
    if (p.kind != SPL_ROW && p.kind != SPL_NNZ && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "unknown schedule kind %d", s->kind);
    int ct = s->col_tile;
    if (!ct) {
        ct = 8;
        while (ct < 64 && ct < N) ct <<= 1;
    }
    if (ct != 8 && ct != 16 && ct != 32 && ct != 64)
        return fail(ctx, SPL_ERR_ARG, "col_tile must be 8, 16, 32 or 64");
    p.col_tile = ct;
    p.items = s->items_per_lane ? s->items_per_lane : 16;
    if (p.items != 8 && p.items != 16 && p.items != 32)
        return fail(ctx, SPL_ERR_ARG, "SpMM items_per_lane must be 8, 16 or 32");
    p.tile = s->tile ? s->tile : (p.kind == SPL_ROW ? 256 / ct : 4 * (256 / ct) * p.items);
    if (p.tile < 1) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    if (s->variant < 0 || s->variant > 2)
        return fail(ctx, SPL_ERR_ARG,
                    "SpMM variant must be 0 (16-byte lanes), 1 (one column per lane) or 2 "
                    "(8-byte BF16 lanes)");
    if (s->variant == 2 && B->vtype != SPL_BF16)
        return fail(ctx, SPL_ERR_ARG, "SpMM variant 2 (8-byte lanes) is for BF16 values");
    p.variant = s->variant;
    return SPL_OK;
}

struct Carved {
    Tiles tiles;
    void *carry;
};

// pos64: the tile positions are int64 (tiles.pos64), else int32 (tiles.pos).
Carved carve(void *ws, int64_t ntiles, bool pos64 = false) {
    char *b = static_cast<char *>(ws);
    Carved c;
    c.tiles.ntiles = ntiles;
    c.tiles.row = reinterpret_cast<int32_t *>(b);
    b += align_up(static_cast<size_t>(ntiles + 1) * 4);
    if (pos64)
        c.tiles.pos64 = reinterpret_cast<int64_t *>(b);
    else
        c.tiles.pos = reinterpret_cast<int32_t *>(b);
    b += align_up(static_cast<size_t>(ntiles + 1) * (pos64 ? 8 : 4));
    c.carry = b;
    return c;
}

// Make `need` bytes of workspace available: the caller's, else the context's.
spl_status get_workspace(spl_context *ctx, void *user, size_t user_bytes, size_t need,
                         void **out) {
    if (need == 0) {
        *out = user;
        return SPL_OK;
    }
    if (user) {
        if (user_bytes < need)
            return fail(ctx, SPL_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", user_bytes,
                        need);
        *out = user;
        return SPL_OK;
    }
    if (ctx->ws_bytes < need) {
        if (ctx->ws) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
            (void)hipFree(ctx->ws);
            ctx->ws = nullptr;
            ctx->ws_bytes = 0;
        }
        size_t sz = std::max(need, static_cast<size_t>(1) << 20);
        if (hipMalloc(&ctx->ws, sz) != hipSuccess) {
            (void)hipGetLastError();
            ctx->ws = nullptr;
            return fail(ctx, SPL_ERR_NOMEM, "hipMalloc(%zu) failed", sz);
        }
        ctx->ws_bytes = sz;
    }
    *out = ctx->ws;
    return SPL_OK;
}

spl_status set_device(spl_context *ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    return SPL_OK;
}

hipEvent_t take_event(spl_context *ctx) {
    if (!ctx->spare.empty()) {
        hipEvent_t e = ctx->spare.back();
        ctx->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets one leaf launch with events when timing is on.
struct LeafTimer {
    spl_context *ctx;
    hipStream_t s;
    int op;
    hipEvent_t a = nullptr, b = nullptr;
    LeafTimer(spl_context *c, int o, hipStream_t st) : ctx(c), s(st), op(o) {
        if (!ctx->timing) return;
        a = take_event(ctx);
        b = take_event(ctx);
        if (a && b) (void)hipEventRecord(a, s);
    }
    void stop() {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        ctx->marks.push_back({a, b, op});
        a = b = nullptr;
    }
};

#define SPL_CHECK(expr)                  \
    do {                                 \
        spl_status _st = (expr);         \
        if (_st != SPL_OK) return _st;   \
    } while (0)

#define SPL_HIP(expr, where)                                   \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
    } while (0)

// Tiled leaf layout: the level partition is cut into pieces (merge split:
// pieces of exactly one chunk of the leaf kernel, so the kernel never
// searches; non-zero split: pieces of T positions), and each workgroup walks
// `stride` consecutive pieces, producing one carry.
struct Pieces {
    int64_t size;     // partition tile size of one piece
    int64_t stride;   // pieces per workgroup
    int64_t count;    // number of pieces
    int64_t blocks;   // workgroups = carries
};

Pieces pieces_for(const Plan &p, int64_t rows, int64_t nnz, int64_t chunk) {
    Pieces q;
    if (p.kind == SPL_MERGE) {
        q.size = chunk;
        q.stride = std::max<int64_t>(1, (p.tile + chunk - 1) / chunk);
    } else {
        q.size = p.tile;
        q.stride = 1;
    }
    q.count = spl::tile_count(p.kind, rows, nnz, q.size);
    q.blocks = (q.count + q.stride - 1) / q.stride;
    return q;
}

// Merged items per leaf chunk: lane groups of one workgroup times the items
// each group walks.
int64_t spmm_chunk(const Plan &p) { return (256 / (p.col_tile / p.vec)) * p.items; }

size_t dtype_bytes(int dt) { return dt == SPL_F64 ? 8 : dt == SPL_F32 ? 4 : 2; }

// Vector lanes for the merge-split SpMM leaf: each lane reads and writes v
// columns with one vector access (variant 0: spl::spmm_vec_width, 16 bytes;
// variant 2: 4 BF16 columns, 8 bytes), when the columns, leading dimensions
// and pointers allow it and a lane group still has 4 to 32 lanes and walks
// 8 or 16 items; otherwise one column per lane.
int spmm_vec(const Plan &p, int vtype, const spl_dense *C, const spl_dense *A) {
    if (p.kind != SPL_MERGE || p.variant == 1 || p.items > 16) return 1;
    const int v = p.variant == 2 ? 4 : spl::spmm_vec_width(vtype);
    const int64_t lanes = p.col_tile / v;
    const int64_t N = C->dims[1];
    const size_t cb = v * dtype_bytes(C->dtype), ab = v * dtype_bytes(A->dtype);
    const bool ok = lanes >= 4 && lanes <= 32 && N % v == 0 && C->ld % v == 0 &&
                    A->ld % v == 0 && reinterpret_cast<uintptr_t>(C->data) % cb == 0 &&
                    reinterpret_cast<uintptr_t>(A->data) % ab == 0;
    return ok ? v : 1;
}

size_t tiled_ws(const Pieces &q, int64_t ncols, size_t elem, size_t pos_bytes = 4) {
    return align_up(static_cast<size_t>(q.count + 1) * 4) +
           align_up(static_cast<size_t>(q.count + 1) * pos_bytes) +
           align_up(static_cast<size_t>(q.blocks) * ncols * elem);
}

size_t spmv_ws(const spl_sparse *B, const Plan &p) {
    if (p.kind == SPL_ROW) return 0;
    return tiled_ws(pieces_for(p, B->dims[0], B->nnz, spmv_chunk(p)), 1, sizeof(double),
                    B->pos_type == SPL_I64 ? 8 : 4);
}

size_t spmm_ws(const spl_sparse *B, int64_t N, const Plan &p) {
    if (p.kind == SPL_ROW) return 0;
    return tiled_ws(pieces_for(p, B->dims[0], B->nnz, spmm_chunk(p)), N,
                    B->vtype == SPL_F64 ? 8 : 4, B->pos_type == SPL_I64 ? 8 : 4);
}

// SpTTV runs the SpMV leaf on the fiber level: a CSR view whose rows are the
// fibers of B (pos = pos[2], crd = crd[2]).
spl_sparse fiber_view(const spl_sparse *B) {
    spl_sparse v = *B;
    v.order = 2;
    v.dims[0] = B->nfibers;
    v.dims[1] = B->dims[2];
    v.dims[2] = 0;
    v.pos[1] = B->pos[2];
    v.crd[1] = B->crd[2];
    v.level[2] = SPL_DENSE;
    return v;
}

// A (Dense, Dense, Compressed) 3-tensor: the middle level is Dense, so slice
// i holds fibers [i J, (i + 1) J) and fiber f has coordinate j = f mod J
// (Sec. III-B, Table I).  The MTTKRP and inner-product leaves walk a
// Compressed middle level; for a Dense one, its pos/crd are written into the
// call's workspace first (I + 1 and I J int32) and the leaves run unchanged.
bool dense_middle(const spl_sparse *B) { return B->order == 3 && B->level[1] == SPL_DENSE; }

size_t dense_middle_ws(const spl_sparse *B) {
    if (!dense_middle(B)) return 0;
    return align_up(static_cast<size_t>(B->dims[0] + 1) * 4) +
           align_up(static_cast<size_t>(B->nfibers) * 4);
}

// A Compressed-middle view of B, whose middle level is expanded at `ws`
// (advanced past it) when it is Dense.
spl_status expand_middle(spl_context *ctx, const spl_sparse *B, char *&ws, spl_sparse &v,
                         hipStream_t s) {
    v = *B;
    if (!dense_middle(B)) return SPL_OK;
    int32_t *pos1 = reinterpret_cast<int32_t *>(ws);
    ws += align_up(static_cast<size_t>(B->dims[0] + 1) * 4);
    int32_t *crd1 = reinterpret_cast<int32_t *>(ws);
    ws += align_up(static_cast<size_t>(B->nfibers) * 4);
    SPL_HIP(spl::launch_dense_level(B->dims[0], B->dims[1], pos1, crd1, s), "dense level launch");
    v.level[1] = SPL_COMPRESSED;
    v.pos[1] = pos1;
    v.crd[1] = crd1;
    return SPL_OK;
}

spl_status resolve_mttkrp(spl_context *ctx, int64_t R, const spl_schedule *s, Plan &p) {
    spl_schedule d{};
    if (!s) s = &d;
    p.kind = s->kind == SPL_SCHED_DEFAULT ? SPL_MERGE : s->kind;
    if (p.kind != SPL_ROW && p.kind != SPL_NNZ && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "unknown schedule kind %d", s->kind);
    int ct = s->col_tile;
    if (!ct) {
        ct = 16;
        while (ct < 64 && ct < R) ct <<= 1;
    }
    if (ct != 16 && ct != 32 && ct != 64)
        return fail(ctx, SPL_ERR_ARG, "MTTKRP col_tile must be 16, 32 or 64");
    p.col_tile = ct;
    // 0: chosen with the lane width (finish_mttkrp)
    p.items = s->items_per_lane;
    if (p.items != 0 && p.items != 3 && p.items != 4 && p.items != 5 && p.items != 8 &&
        p.items != 16)
        return fail(ctx, SPL_ERR_ARG, "MTTKRP items_per_lane must be 3, 4, 5, 8 or 16");
    p.tile = s->tile;  // 0: chosen with the lane width
    if (p.tile < 0) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    if (s->variant < 0 || s->variant > 3)
        return fail(ctx, SPL_ERR_ARG,
                    "MTTKRP variant must be 0 (vector lanes), 1 (one column per lane), 2 "
                    "(8-byte BF16 lanes) or 3 (FP32 vector lanes with positions staged in LDS)");
    p.variant = s->variant;
    return SPL_OK;
}

// Merged items per leaf chunk: lane groups of one workgroup (128 threads for
// the vector-lane leaf, 256 for one column per lane) times items per group.
int64_t mttkrp_chunk(const Plan &p) {
    const int64_t threads = p.vec > 1 ? spl::kMttkrpThreads : 256;
    return (threads / (p.col_tile / p.vec)) * p.items;
}

// The defaults that depend on the lane width p.vec: items per lane group
// (5 for 8 lanes of 4 columns, 3 for 4 lanes of 8 BF16 columns -- each the
// most merged items whose registers still leave 4 waves per SIMD; 4 for the
// other vector lanes and for variant 3; 8 for one column per lane) and the
// tile (512 merged items with vector lanes, four 256-thread chunks
// otherwise).  With int64 positions the 4-column leaf takes 4 items: 5 would
// need one register more than 4 waves per SIMD allow.
void finish_mttkrp(Plan &p, bool pos64) {
    const int lanes = p.col_tile / p.vec;
    if (p.items == 0) {
        if (p.vec == 1)
            p.items = 8;
        else if (p.variant == 3)
            p.items = 4;
        else if (p.vec == 8)
            p.items = lanes == 4 ? 3 : 4;
        else
            p.items = lanes == 8 && !pos64 ? 5 : 4;
    }
    if (p.tile == 0)
        p.tile = p.kind == SPL_ROW ? 64 : p.kind == SPL_NNZ ? 2048
                 : p.vec > 1     ? 512
                                 : 4 * mttkrp_chunk(p);
}

// Vector lanes for the MTTKRP leaf: v rank columns per lane when R, the
// leading dimensions and the pointers allow it, col_tile is 32 or 64 and
// items_per_lane is not 16; otherwise one column per lane.  v = 4 (16-byte
// FP32 rows, 8-byte BF16 rows; BF16 variant 2), or for BF16 under variant 0
// v = 8 (16-byte rows) with (col_tile, items) (32, 3), (32, 4), (64, 4),
// (64, 8) or items chosen by default.
int mttkrp_vec(const Plan &p, const spl_dense *C, const spl_dense *D, const spl_dense *A) {
    if (p.variant == 1 || p.items == 16 || (p.col_tile != 32 && p.col_tile != 64)) return 1;
    const int64_t R = C->dims[1];
    auto fits = [&](int v) {
        const size_t fb = v * dtype_bytes(C->dtype);
        return R % v == 0 && C->ld % v == 0 && D->ld % v == 0 && A->ld % v == 0 &&
               reinterpret_cast<uintptr_t>(C->data) % fb == 0 &&
               reinterpret_cast<uintptr_t>(D->data) % fb == 0 &&
               reinterpret_cast<uintptr_t>(A->data) % 16 == 0;
    };
    const bool bf = C->dtype == SPL_BF16;
    if (bf && p.variant == 0 && fits(8) &&
        (p.items == 0 || p.items == 4 || (p.items == 3 && p.col_tile == 32) ||
         (p.items == 8 && p.col_tile == 64)))
        return 8;
    return fits(4) ? 4 : 1;
}

// MTTKRP pieces live in (slice, fiber) coordinates.
Pieces mttkrp_pieces(const spl_sparse *B, const Plan &p) {
    Pieces q = pieces_for(p, B->dims[0], B->nfibers, mttkrp_chunk(p));
    if (p.kind == SPL_NNZ) {
        q.count = spl::tile_count(SPL_NNZ, 0, B->nnz, p.tile);
        q.blocks = q.count;
    }
    return q;
}

size_t mttkrp_ws(const spl_sparse *B, int64_t R, const Plan &p) {
    return tiled_ws(mttkrp_pieces(B, p), R, sizeof(float));
}

spl_status resolve_sddmm(spl_context *ctx, const spl_schedule *s, Plan &p) {
    spl_schedule d{};
    if (!s) s = &d;
    p.kind = s->kind == SPL_SCHED_DEFAULT ? SPL_MERGE : s->kind;
    if (p.kind != SPL_ROW && p.kind != SPL_NNZ && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "unknown schedule kind %d", s->kind);
    // default merge tile: one chunk per workgroup for the vector leaf (more
    // workgroups in flight: FP32 0.87 against 1.04 ms with four chunks at
    // K = 128), four for the matrix-core leaf
    const int64_t merge_tile = (s->variant == 1 ? 4 : 1) * spl::sddmm_chunk();
    p.tile = s->tile ? s->tile
                     : (p.kind == SPL_ROW ? 64 : p.kind == SPL_NNZ ? 1024 : merge_tile);
    if (p.tile < 1) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    p.items = s->variant;
    return SPL_OK;
}

size_t sddmm_ws(const spl_sparse *B, const Plan &p) {
    return tiled_ws(pieces_for(p, B->dims[0], B->nnz, spl::sddmm_chunk()), 0, 1);
}

constexpr int64_t kInnerParts = 2048;

// Workspace of an inner product with B as the first operand: the shared-
// pattern partials or the general co-iteration's per-workgroup partials.
size_t inner_ws(const spl_sparse *B) {
    const int64_t units = B->order == 2 ? B->nnz : B->nfibers;
    return align_up(std::max(static_cast<size_t>(kInnerParts) * sizeof(double),
                             spl::inner_general_ws(units)));
}

size_t spadd3_ws(int64_t n) {
    return align_up(static_cast<size_t>(spl::spadd3_scan_tiles(n)) * 8) + align_up(8);
}

bool same_dims(const spl_sparse *a, const spl_sparse *b) {
    for (int l = 0; l < a->order; ++l)
        if (a->dims[l] != b->dims[l]) return false;
    return true;
}

// ------------------------------------------------------------- TIN parse
// Canonical form: white space removed, every tensor name replaced by 'T'
// and index variables renamed a, b, c, ... in order of first appearance.
bool canonical(const char *in, std::string &out) {
    std::string s;
    for (const char *c = in; *c; ++c)
        if (!std::isspace(static_cast<unsigned char>(*c))) s += *c;
    std::string res, names;
    bool inside = false;
    size_t i = 0;
    while (i < s.size()) {
        char c = s[i];
        if (std::isalpha(static_cast<unsigned char>(c)) || c == '_') {
            size_t j = i;
            while (j < s.size() && (std::isalnum(static_cast<unsigned char>(s[j])) || s[j] == '_')) ++j;
            std::string tok = s.substr(i, j - i);
            if (inside) {
                // index variable
                size_t k = 0;
                std::string key = "|" + tok + "|";
                size_t at = names.find(key);
                if (at == std::string::npos) {
                    int count = 0;
                    for (char ch : names) count += ch == '|';
                    names += key;
                    k = static_cast<size_t>(count / 2);
                } else {
                    int count = 0;
                    for (size_t q = 0; q < at; ++q) count += names[q] == '|';
                    k = static_cast<size_t>(count / 2);
                }
                res += static_cast<char>('a' + k);
            } else {
                res += 'T';
            }
            i = j;
            continue;
        }
        if (c == '(') inside = true;
        if (c == ')') inside = false;
        if (std::strchr("()=*+,", c) == nullptr) return false;
        res += c;
        ++i;
    }
    out = res;
    return true;
}

const char *const kTin[7] = {
    "a(i)=B(i,j)*c(j)",
    "A(i,j)=B(i,k)*C(k,j)",
    "A(i,j)=B(i,j)+C(i,j)+D(i,j)",
    "A(i,j)=B(i,j)*C(i,k)*D(j,k)",
    "A(i,j)=B(i,j,k)*c(k)",
    "A(i,l)=B(i,j,k)*C(j,l)*D(k,l)",
    "a=B(i,j,k)*C(i,j,k)",
};

spl_schedule make_sched(int kind, int lanes, int tile, int items, int col_tile) {
    spl_schedule s{};
    s.kind = kind;
    s.lanes_per_row = lanes;
    s.tile = tile;
    s.items_per_lane = items;
    s.col_tile = col_tile;
    return s;
}

// The library's candidate lists for spl_autotune and SPL_SCHED_AUTOTUNE:
// SpMV row splits of 1..64 lanes, non-zero splits of 1024..4096 positions
// and two merge splits; SpMM row split and non-zero/merge splits at 32
// columns per lane group.
const std::vector<spl_schedule> &default_candidates(spl_op op) {
    static const std::vector<spl_schedule> spmv = [] {
        std::vector<spl_schedule> v;
        for (int L : {1, 2, 4, 8, 16, 32, 64}) v.push_back(make_sched(SPL_ROW, L, 0, 0, 0));
        for (int T : {1024, 2048, 4096}) v.push_back(make_sched(SPL_NNZ, 0, T, 8, 0));
        v.push_back(make_sched(SPL_MERGE, 0, 1024, 4, 0));
        v.push_back(make_sched(SPL_MERGE, 0, 2048, 8, 0));
        return v;
    }();
    static const std::vector<spl_schedule> spmm = [] {
        std::vector<spl_schedule> v;
        v.push_back(make_sched(SPL_ROW, 0, 0, 0, 32));
        for (int T : {256, 1024}) v.push_back(make_sched(SPL_NNZ, 0, T, 16, 32));
        for (int it : {8, 16, 32})
            for (int k : {1, 4}) v.push_back(make_sched(SPL_MERGE, 0, 8 * it * k, it, 32));
        return v;
    }();
    return op == SPL_OP_SPMV ? spmv : spmm;
}

int sel_index(spl_op op) { return op == SPL_OP_SPMV ? 0 : op == SPL_OP_SPMM ? 1 : -1; }

bool concrete_kind(int k) { return k >= SPL_SCHED_DEFAULT && k <= SPL_MERGE; }

bool selection_kind(const spl_schedule *s) {
    return s && (s->kind == SPL_SCHED_LEARNED || s->kind == SPL_SCHED_AUTOTUNE);
}

// The schedules a selection kind chooses among: the installed selector's
// candidates (SPL_SCHED_LEARNED needs one; SPL_SCHED_AUTOTUNE uses them when
// present), else the library's list.
spl_status selection_candidates(spl_context *ctx, spl_op op, int kind,
                                const std::vector<spl_schedule> *&out) {
    const int i = sel_index(op);
    if (i < 0)
        return fail(ctx, SPL_ERR_UNSUPPORTED, "learned and autotuned schedules cover SpMV and SpMM");
    if (ctx->sel[i].K > 0) {
        out = &ctx->sel[i].cands;
        return SPL_OK;
    }
    if (kind == SPL_SCHED_LEARNED)
        return fail(ctx, SPL_ERR_UNSUPPORTED, "no schedule selector installed (spl_mlp_load)");
    out = &default_candidates(op);
    return SPL_OK;
}

// Events of one autotuning run, destroyed on every exit path.
struct EventSet {
    std::vector<hipEvent_t> e;
    explicit EventSet(int n) : e(n, nullptr) {}
    ~EventSet() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Resolve SPL_SCHED_LEARNED / SPL_SCHED_AUTOTUNE to one concrete schedule
// (`chosen`, which `sched` then points to); other kinds pass through.
spl_status select_schedule(spl_context *ctx, spl_op op, const spl_sparse *B, const spl_dense *X,
                           spl_dense *Y, const spl_schedule *&sched, spl_schedule &chosen,
                           spl_stream stream) {
    if (!selection_kind(sched)) return SPL_OK;
    if (sched->kind == SPL_SCHED_LEARNED) {
        SPL_CHECK(spl_mlp_predict(ctx, op, B, &chosen, stream));
    } else {
        const std::vector<spl_schedule> *c = nullptr;
        SPL_CHECK(selection_candidates(ctx, op, SPL_SCHED_AUTOTUNE, c));
        SPL_CHECK(spl_autotune(ctx, op, B, X, Y, c->data(), static_cast<int>(c->size()), 3,
                               &chosen, nullptr, stream));
    }
    sched = &chosen;
    return SPL_OK;
}

// Bindings of one index-notation call, its plan for this call's operands,
// and the compiled leaves for those formats (from the context's cache, or
// generated and compiled now when `compile` is set).
spl_status tin_prepare(spl_context *ctx, const char *stmt, int nops, const spl_tin_operand *ops,
                       const spl_tin_operand *out, std::vector<spl::tin::Binding> &b,
                       spl::tin::Binding &ob, spl::tin::Program &prog,
                       spl::tin::Program **compiled) {
    if (!stmt || !out || nops < 0 || (nops > 0 && !ops))
        return fail(ctx, SPL_ERR_ARG, "NULL statement, operand list or output");
    b.resize(static_cast<size_t>(nops));
    for (int k = 0; k < nops; ++k) {
        if (!ops[k].name) return fail(ctx, SPL_ERR_ARG, "operand %d has no name", k);
        b[k].name = ops[k].name;
        b[k].sparse = ops[k].sparse;
        b[k].dense = ops[k].dense;
    }
    if (!out->name) return fail(ctx, SPL_ERR_ARG, "the output has no name");
    ob.name = out->name;
    ob.sparse = out->sparse;
    ob.dense = out->dense;
    std::string err;
    spl_status st = spl::tin::plan(stmt, b, ob, prog, err);
    if (st != SPL_OK) return fail(ctx, st, "%s", err.c_str());
    if (!compiled) return SPL_OK;
    auto it = ctx->tin_cache.find(prog.key);
    if (it == ctx->tin_cache.end()) {
        SPL_CHECK(set_device(ctx));
        std::unique_ptr<spl::tin::Program> c(new spl::tin::Program(prog));
        st = spl::tin::compile(*c, err);
        if (st != SPL_OK) return fail(ctx, st, "%s", err.c_str());
        it = ctx->tin_cache.emplace(prog.key, std::move(c)).first;
    }
    *compiled = it->second.get();
    return SPL_OK;
}

hipError_t tin_launch(hipFunction_t f, int64_t rows, std::vector<unsigned long long> &slots,
                      hipStream_t s) {
    if (rows == 0) return hipSuccess;
    void *args[] = {slots.data()};
    return hipModuleLaunchKernel(f, static_cast<unsigned>((rows + 255) / 256), 1, 1, 256, 1, 1,
                                 0, s, args, nullptr);
}

}  // namespace

extern "C" {

const char *spl_status_string(spl_status s) {
    switch (s) {
    case SPL_OK: return "SPL_OK";
    case SPL_ERR_ARG: return "SPL_ERR_ARG";
    case SPL_ERR_FORMAT: return "SPL_ERR_FORMAT";
    case SPL_ERR_SHAPE: return "SPL_ERR_SHAPE";
    case SPL_ERR_DTYPE: return "SPL_ERR_DTYPE";
    case SPL_ERR_UNSUPPORTED: return "SPL_ERR_UNSUPPORTED";
    case SPL_ERR_WORKSPACE: return "SPL_ERR_WORKSPACE";
    case SPL_ERR_NOMEM: return "SPL_ERR_NOMEM";
    case SPL_ERR_HIP: return "SPL_ERR_HIP";
    case SPL_ERR_INVALID: return "SPL_ERR_INVALID";
    }
    return "unknown status";
}

spl_status spl_context_create(int device, spl_context **out) {
    spl_context *ctx = nullptr;
    SPL_GUARD_BEGIN
    if (!out) return SPL_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return SPL_ERR_ARG;
    }
    ctx = new spl_context();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&ctx->flags), 2 * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&ctx->readback), 2 * sizeof(int64_t),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->flags) (void)hipFree(ctx->flags);
        delete ctx;
        return SPL_ERR_HIP;
    }
    // device address of this GPU's static scratch (spl_spmv_noalloc); a
    // failure is kept and reported by that call only
    ctx->scratch_status = spl::scratch_init(device);
    *out = ctx;
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_context_destroy(spl_context *ctx) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->flags) (void)hipFree(ctx->flags);
    if (ctx->readback) (void)hipHostFree(ctx->readback);
    for (const auto &m : ctx->marks) {
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
    for (auto &sl : ctx->sel)
        for (float *b : {sl.params, sl.norm, sl.m, sl.v, sl.scratch})
            if (b) (void)hipFree(b);
    ctx->tin_cache.clear();  // unloads the generated modules on this device
    delete ctx;
    return SPL_OK;
    SPL_GUARD_END
}

const char *spl_last_error(const spl_context *ctx) { return ctx ? ctx->err.c_str() : ""; }

spl_status spl_timing_enable(spl_context *ctx, int enable) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    ctx->timing = enable != 0;
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_timing_read(spl_context *ctx, spl_op op, int64_t *launches, double *total_ms) {
    SPL_GUARD_BEGIN
    if (!ctx || !launches || !total_ms) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    SPL_CHECK(set_device(ctx));
    int64_t count = 0;
    double sum = 0.0;
    std::vector<spl_context::Mark> keep;
    spl_status st = SPL_OK;
    for (const auto &m : ctx->marks) {
        if (m.op != op) {
            keep.push_back(m);
            continue;
        }
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(m.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.start, m.stop);
        if (e != hipSuccess && st == SPL_OK) st = hip_fail(ctx, e, "hipEventElapsedTime");
        sum += ms;
        ++count;
        ctx->spare.push_back(m.start);
        ctx->spare.push_back(m.stop);
    }
    ctx->marks.swap(keep);
    *launches = count;
    *total_ms = sum;
    return st;
    SPL_GUARD_END
}

spl_status spl_sync(spl_context *ctx, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(set_device(ctx));
    SPL_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    return SPL_OK;
    SPL_GUARD_END
}

const char *spl_op_tin(spl_op op) {
    if (op < SPL_OP_SPMV || op > SPL_OP_INNER) return nullptr;
    return kTin[op];
}

spl_status spl_op_parse(const char *tin, spl_op *out) {
    spl_context *ctx = nullptr;
    SPL_GUARD_BEGIN
    if (!tin || !out) return SPL_ERR_ARG;
    std::string got;
    if (!canonical(tin, got)) return SPL_ERR_UNSUPPORTED;
    for (int k = 0; k < 7; ++k) {
        std::string ref;
        canonical(kTin[k], ref);
        // a scalar output may be written with empty parentheses
        std::string alt = ref;
        if (k == SPL_OP_INNER) alt = "T()" + ref.substr(1);
        if (got == ref || got == alt) {
            *out = static_cast<spl_op>(k);
            return SPL_OK;
        }
    }
    return SPL_ERR_UNSUPPORTED;
    SPL_GUARD_END
}

spl_status spl_workspace_query(spl_context *ctx, spl_op op, const spl_sparse *B, int64_t ncols,
                               const spl_schedule *sched, size_t *bytes) {
    SPL_GUARD_BEGIN
    if (!ctx || !bytes) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    *bytes = 0;
    Plan p;
    switch (op) {
    case SPL_OP_SPMV:
    case SPL_OP_SPMM: {
        SPL_CHECK(check_sparse(ctx, B, 2, true));
        // a selection kind needs room for whichever candidate it picks
        std::vector<spl_schedule> one;
        const std::vector<spl_schedule> *list = &one;
        if (selection_kind(sched))
            SPL_CHECK(selection_candidates(ctx, op, sched->kind, list));
        else
            one.push_back(sched ? *sched : spl_schedule{});
        for (const spl_schedule &c : *list) {
            if (op == SPL_OP_SPMV) {
                SPL_CHECK(resolve_spmv(ctx, B, &c, p));
                *bytes = std::max(*bytes, spmv_ws(B, p));
            } else {
                SPL_CHECK(resolve_spmm(ctx, B, ncols, &c, p));
                *bytes = std::max(*bytes, spmm_ws(B, ncols, p));
            }
        }
        return SPL_OK;
    }
    case SPL_OP_SPTTV: {
        SPL_CHECK(check_sparse(ctx, B, 3, true));
        const spl_sparse v = fiber_view(B);
        SPL_CHECK(resolve_spmv(ctx, &v, sched, p));
        *bytes = spmv_ws(&v, p);
        return SPL_OK;
    }
    case SPL_OP_MTTKRP: {
        SPL_CHECK(check_sparse(ctx, B, 3, true));
        SPL_CHECK(resolve_mttkrp(ctx, ncols, sched, p));
        // the lane width depends on the factors' pointers: the largest
        // workspace over every width the call may take
        size_t ws = 0;
        for (int v : {1, 4, 8}) {
            Plan q = p;
            q.vec = v;
            finish_mttkrp(q, B->pos_type == SPL_I64);
            ws = std::max(ws, mttkrp_ws(B, ncols, q));
        }
        *bytes = dense_middle_ws(B) + ws;
        return SPL_OK;
    }
    case SPL_OP_SDDMM:
        SPL_CHECK(check_sparse(ctx, B, 2));
        SPL_CHECK(resolve_sddmm(ctx, sched, p));
        *bytes = sddmm_ws(B, p);
        return SPL_OK;
    case SPL_OP_INNER:
        if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
        if (B->order != 2 && B->order != 3) return fail(ctx, SPL_ERR_FORMAT, "order must be 2 or 3");
        SPL_CHECK(check_sparse(ctx, B, B->order));
        *bytes = dense_middle_ws(B) + inner_ws(B);
        return SPL_OK;
    case SPL_OP_SPADD3:
        SPL_CHECK(check_sparse(ctx, B, 2));
        *bytes = spadd3_ws(B->dims[0]);
        return SPL_OK;
    default:
        return fail(ctx, SPL_ERR_UNSUPPORTED, "op %d has no workspace query yet", op);
    }
    SPL_GUARD_END
}

spl_status spl_tile_bounds(spl_context *ctx, const spl_sparse *B, const spl_schedule *sched,
                           int32_t *tile_row, int32_t *tile_pos, int64_t capacity,
                           int64_t *ntiles, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
    SPL_CHECK(check_sparse(ctx, B, B->order == 3 ? 3 : 2));
    if (!sched || !tile_row || !tile_pos || !ntiles)
        return fail(ctx, SPL_ERR_ARG, "NULL argument");
    const int kind = sched->kind;
    if (kind != SPL_ROW && kind != SPL_NNZ && kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_ARG, "tile bounds need kind ROW, NNZ or MERGE");
    if (sched->tile < 1) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    const int last = B->order - 1;
    const int64_t rows = B->order == 3 ? B->nfibers : B->dims[0];
    const int64_t nt = spl::tile_count(kind, rows, B->nnz, sched->tile);
    *ntiles = nt;
    if (capacity < nt + 1)
        return fail(ctx, SPL_ERR_ARG, "capacity %lld < %lld tile bounds",
                    static_cast<long long>(capacity), static_cast<long long>(nt + 1));
    SPL_CHECK(set_device(ctx));
    Tiles t{tile_row, tile_pos, nt};
    SPL_HIP(spl::launch_tile_bounds(kind, rows, B->pos[last], B->nnz, sched->tile, t,
                                    static_cast<hipStream_t>(stream)),
            "tile bounds launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_csf_tile_bounds(spl_context *ctx, const spl_sparse *B, int64_t T,
                               int32_t *tile_slice, int32_t *tile_fiber, int64_t capacity,
                               int64_t *ntiles, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 3));
    if (dense_middle(B))
        return fail(ctx, SPL_ERR_FORMAT, "CSF tile bounds need a Compressed middle level");
    if (!tile_slice || !tile_fiber || !ntiles) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    if (T < 1) return fail(ctx, SPL_ERR_ARG, "T must be positive");
    const int64_t nt = spl::tile_count(SPL_NNZ, 0, B->nnz, T);
    *ntiles = nt;
    if (capacity < nt + 1)
        return fail(ctx, SPL_ERR_ARG, "capacity %lld < %lld tile bounds",
                    static_cast<long long>(capacity), static_cast<long long>(nt + 1));
    SPL_CHECK(set_device(ctx));
    Tiles t{tile_slice, tile_fiber, nt};
    SPL_HIP(spl::launch_csf_nnz_bounds(B->dims[0], B->pos[1], B->nfibers, B->pos[2], B->nnz, T, t,
                                       static_cast<hipStream_t>(stream)),
            "CSF bounds launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_validate(spl_context *ctx, const spl_sparse *B, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
    SPL_CHECK(check_sparse(ctx, B, B->order == 3 ? 3 : 2));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = dense_middle(B) ? 2 : 1; l < B->order; ++l) {
        const int64_t parents = l == 1 ? B->dims[0] : B->nfibers;
        const int64_t children = l == B->order - 1 ? B->nnz : B->nfibers;
        const int64_t extent = B->dims[l];
        const int64_t init[2] = {0, -1};
        SPL_HIP(hipMemcpyAsync(ctx->flags, init, sizeof init, hipMemcpyHostToDevice, s),
                "hipMemcpyAsync");
        SPL_HIP(spl::launch_validate_level(parents, B->pos[l], B->crd[l], children, extent,
                                           ctx->flags, s),
                "validate launch");
        SPL_HIP(hipMemcpyAsync(ctx->readback, ctx->flags, 2 * sizeof(int64_t),
                               hipMemcpyDeviceToHost, s),
                "hipMemcpyAsync");
        SPL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        const int64_t res[2] = {ctx->readback[0], ctx->readback[1]};
        if (res[0] != 0) {
            const unsigned code = static_cast<unsigned>(res[0]);
            const char *what = (code & 1u)    ? "pos[0] != 0"
                               : (code & 2u)  ? "pos decreases"
                               : (code & 4u)  ? "last pos != child count"
                               : (code & 8u)  ? "crd out of range"
                                              : "crd not strictly increasing";
            return fail(ctx, SPL_ERR_INVALID, "level %d: %s (first at parent %lld)", l, what,
                        static_cast<long long>(res[1]));
        }
    }
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_probe(spl_context *ctx, int kind, const void *buf, int64_t bytes,
                     int64_t row_bytes, int64_t count, double *out, int64_t blocks,
                     spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!buf || !out) return fail(ctx, SPL_ERR_ARG, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0)
        return fail(ctx, SPL_ERR_ARG, "buffer must be 16-byte aligned");
    if (blocks < 1 || blocks > (1LL << 31) - 1) return fail(ctx, SPL_ERR_ARG, "bad block count");
    if (kind == 0) {
        if (bytes < 16 || bytes % 16 != 0)
            return fail(ctx, SPL_ERR_ARG, "stream probe needs a positive multiple of 16 bytes");
    } else if (kind == 1) {
        if (row_bytes != 4 && row_bytes != 8 && row_bytes != 32 && row_bytes != 64 &&
            row_bytes != 128 && row_bytes != 256)
            return fail(ctx, SPL_ERR_ARG, "row_bytes must be 4, 8, 32, 64, 128 or 256");
        if (bytes < row_bytes || count < 0) return fail(ctx, SPL_ERR_ARG, "bad table or count");
    } else if (kind == 2) {
        if (row_bytes != 16 && row_bytes != 64 && row_bytes != 128 && row_bytes != 256)
            return fail(ctx, SPL_ERR_ARG, "row_bytes must be 16, 64, 128 or 256");
        if (bytes < row_bytes || count < 0) return fail(ctx, SPL_ERR_ARG, "bad table or count");
    } else {
        return fail(ctx, SPL_ERR_ARG, "unknown probe kind %d", kind);
    }
    SPL_CHECK(set_device(ctx));
    SPL_HIP(spl::launch_probe(kind, buf, bytes, row_bytes, count, out, blocks,
                              static_cast<hipStream_t>(stream)),
            "probe launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spmv(spl_context *ctx, const spl_sparse *B, const spl_dense *c, spl_dense *a,
                    const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                    spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2, true));
    SPL_CHECK(check_dense(ctx, c, "c", 1, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, a, "a", 1, B->dims[0], -1));
    if (B->vtype == SPL_BF16 || c->dtype != B->vtype || a->dtype != B->vtype)
        return fail(ctx, SPL_ERR_DTYPE, "SpMV needs vals, c and a all F64 or all F32");
    const bool pos64 = B->pos_type == SPL_I64;
    if (pos64 && selection_kind(sched))
        return fail(ctx, SPL_ERR_UNSUPPORTED, "int64 positions: MERGE schedules only");
    spl_schedule chosen{};
    SPL_CHECK(select_schedule(ctx, SPL_OP_SPMV, B, c, a, sched, chosen, stream));
    Plan p;
    SPL_CHECK(resolve_spmv(ctx, B, sched, p));
    if (pos64 && (p.kind != SPL_MERGE || p.variant != 0))
        return fail(ctx, SPL_ERR_UNSUPPORTED, "int64 positions: MERGE schedule, variant 0 only");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    if (n == 0) return SPL_OK;
    if (p.kind == SPL_ROW) {
        LeafTimer tm(ctx, SPL_OP_SPMV, s);
        SPL_HIP(spl::launch_spmv_row(B->vtype, p.lanes, n, B->pos[1], nullptr, B->crd[1], B->vals, c->data,
                                     a->data, s),
                "SpMV row launch");
        tm.stop();
        return SPL_OK;
    }
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmv_ws(B, p), &ws));
    const Pieces q = pieces_for(p, n, B->nnz, spmv_chunk(p));
    Carved cv = carve(ws, q.count, pos64);
    if (pos64) {
        const int64_t *pos = reinterpret_cast<const int64_t *>(B->pos[1]);
        SPL_HIP(spl::launch_merge_bounds64(n, pos, B->nnz, q.size, cv.tiles, s),
                "tile bounds launch");
        LeafTimer tm(ctx, SPL_OP_SPMV, s);
        SPL_HIP(spl::launch_spmv_flag64(B->vtype, p.items, n, pos, B->crd[1], B->vals, c->data,
                                        a->data, cv.tiles, q.stride,
                                        static_cast<double *>(cv.carry), s),
                "SpMV tile launch");
        tm.stop();
        SPL_HIP(spl::launch_spmv_fixup(B->vtype, n, cv.tiles, q.stride,
                                       static_cast<double *>(cv.carry), a->data, s),
                "SpMV fix-up launch");
        return SPL_OK;
    }
    SPL_HIP(spl::launch_tile_bounds(p.kind, n, B->pos[1], B->nnz, q.size, cv.tiles, s),
            "tile bounds launch");
    LeafTimer tm(ctx, SPL_OP_SPMV, s);
    SPL_HIP(spl::launch_spmv_tiles(B->vtype, p.items, n, B->pos[1], B->crd[1], B->vals, c->data,
                                   a->data, cv.tiles, q.stride, /*exact_chunks=*/p.kind == SPL_MERGE,
                                   p.variant, static_cast<double *>(cv.carry), s),
            "SpMV tile launch");
    tm.stop();
    SPL_HIP(spl::launch_spmv_fixup(B->vtype, n, cv.tiles, q.stride,
                                   static_cast<double *>(cv.carry), a->data, s),
            "SpMV fix-up launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spmv_noalloc(spl_context *ctx, const spl_sparse *B, const spl_dense *c,
                            spl_dense *a, const spl_schedule *sched, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (selection_kind(sched))
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "spl_spmv_noalloc: learned and autotuned schedules need the context's "
                    "workspace; pass a ROW, NNZ or MERGE schedule");
    if (ctx->scratch_status != hipSuccess)
        return hip_fail(ctx, ctx->scratch_status, "spl_spmv_noalloc: static scratch lookup");
    void *ptr = spl::scratch_ptr(ctx->device);
    if (!ptr) return fail(ctx, SPL_ERR_HIP, "spl_spmv_noalloc: no static scratch on this device");
    size_t need = 0;
    SPL_CHECK(spl_workspace_query(ctx, SPL_OP_SPMV, B, 1, sched, &need));
    if (need > spl::kScratchBytes)
        return fail(ctx, SPL_ERR_WORKSPACE,
                    "spl_spmv_noalloc: this matrix and schedule need %zu bytes of tile bounds "
                    "and carries; the static scratch holds %zu (use spl_spmv with a workspace, "
                    "or a longer tile)",
                    need, spl::kScratchBytes);
    // leaf timing would create events: off for this call
    const bool timing = ctx->timing;
    ctx->timing = false;
    const spl_status st = spl_spmv(ctx, B, c, a, sched, ptr, spl::kScratchBytes, stream);
    ctx->timing = timing;
    return st;
    SPL_GUARD_END
}

spl_status spl_spmm(spl_context *ctx, const spl_sparse *B, const spl_dense *C, spl_dense *A,
                    const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                    spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2, true));
    if (!C) return fail(ctx, SPL_ERR_ARG, "dense operand C is NULL");
    const bool pos64 = B->pos_type == SPL_I64;
    if (pos64 && selection_kind(sched))
        return fail(ctx, SPL_ERR_UNSUPPORTED, "int64 positions: MERGE schedules only");
    const int64_t N = C->ndim == 2 ? C->dims[1] : -1;
    SPL_CHECK(check_dense(ctx, C, "C", 2, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, A, "A", 2, B->dims[0], N));
    const bool ok = (B->vtype == SPL_F64 && C->dtype == SPL_F64 && A->dtype == SPL_F64) ||
                    (B->vtype == SPL_F32 && C->dtype == SPL_F32 && A->dtype == SPL_F32) ||
                    (B->vtype == SPL_BF16 && C->dtype == SPL_BF16 && A->dtype == SPL_F32);
    if (!ok)
        return fail(ctx, SPL_ERR_DTYPE,
                    "SpMM dtypes (vals, C, A) must be (F64,F64,F64), (F32,F32,F32) or (BF16,BF16,F32)");
    spl_schedule chosen{};
    SPL_CHECK(select_schedule(ctx, SPL_OP_SPMM, B, C, A, sched, chosen, stream));
    Plan p;
    SPL_CHECK(resolve_spmm(ctx, B, N, sched, p));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    if (n == 0 || N == 0) return SPL_OK;
    if (pos64 && p.kind != SPL_MERGE)
        return fail(ctx, SPL_ERR_UNSUPPORTED, "int64 positions: MERGE schedule only");
    if (p.kind == SPL_ROW) {
        LeafTimer tm(ctx, SPL_OP_SPMM, s);
        SPL_HIP(spl::launch_spmm_row(B->vtype, A->dtype, p.col_tile, n, N, B->pos[1], B->crd[1],
                                     B->vals, C->data, C->ld, A->data, A->ld, s),
                "SpMM row launch");
        tm.stop();
        return SPL_OK;
    }
    // the workspace query assumed one column per lane: the larger size
    p.vec = spmm_vec(p, B->vtype, C, A);
    if (pos64 && p.vec != spl::spmm_vec_width(B->vtype))
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "int64 positions: 16-byte vector lanes only (variant 0; N, every ld and the "
                    "dense pointers aligned to 16 bytes; items_per_lane 8 or 16)");
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmm_ws(B, N, p), &ws));
    const Pieces q = pieces_for(p, n, B->nnz, spmm_chunk(p));
    Carved cv = carve(ws, q.count, pos64);
    // branch-free row gathers when C's rows span at most a descriptor's range
    const bool buf = static_cast<double>(C->dims[0]) * static_cast<double>(C->ld) *
                         static_cast<double>(dtype_bytes(C->dtype)) <=
                     spl::kBufRange;
    if (pos64) {
        const int64_t *pos = reinterpret_cast<const int64_t *>(B->pos[1]);
        SPL_HIP(spl::launch_merge_bounds64(n, pos, B->nnz, q.size, cv.tiles, s),
                "tile bounds launch");
        LeafTimer tm(ctx, SPL_OP_SPMM, s);
        SPL_HIP(spl::launch_spmm_tiles64(B->vtype, p.col_tile, p.items, p.vec, n, N, pos,
                                         B->crd[1], B->vals, C->data, C->ld, A->data, A->ld,
                                         cv.tiles, q.stride, buf, cv.carry, s),
                "SpMM tile launch");
        tm.stop();
        SPL_HIP(spl::launch_spmm_fixup(B->vtype, n, N, cv.tiles, q.stride, cv.carry, A->data,
                                       A->ld, s),
                "SpMM fix-up launch");
        return SPL_OK;
    }
    SPL_HIP(spl::launch_tile_bounds(p.kind, n, B->pos[1], B->nnz, q.size, cv.tiles, s),
            "tile bounds launch");
    LeafTimer tm(ctx, SPL_OP_SPMM, s);
    SPL_HIP(spl::launch_spmm_tiles(B->vtype, p.col_tile, p.items, p.vec, n, N, B->pos[1], B->crd[1],
                                   B->vals, C->data, C->ld, A->data, A->ld, cv.tiles, q.stride,
                                   /*exact_chunks=*/p.kind == SPL_MERGE, buf, cv.carry, s),
            "SpMM tile launch");
    tm.stop();
    SPL_HIP(spl::launch_spmm_fixup(B->vtype, n, N, cv.tiles, q.stride, cv.carry, A->data, A->ld,
                                   s),
            "SpMM fix-up launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_coord_partition(spl_context *ctx, const spl_sparse *B, int32_t ncolors,
                               const int32_t *bounds, int32_t *out, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    if (ncolors < 1) return fail(ctx, SPL_ERR_ARG, "ncolors must be at least 1");
    const int64_t n = B->dims[0];
    if (n == 0) return SPL_OK;
    if (!bounds || !out) return fail(ctx, SPL_ERR_ARG, "NULL bounds or output");
    SPL_CHECK(set_device(ctx));
    SPL_HIP(spl::launch_coord_split(n, B->pos[1], B->crd[1], static_cast<int64_t>(ncolors) + 1,
                                    bounds, out, static_cast<hipStream_t>(stream)),
            "coordinate partition launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spmv_window(spl_context *ctx, const spl_sparse *B, const int32_t *begin,
                           const int32_t *end, const spl_dense *c, spl_dense *a,
                           const spl_schedule *sched, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    SPL_CHECK(check_dense(ctx, c, "c", 1, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, a, "a", 1, B->dims[0], -1));
    if (B->vtype == SPL_BF16 || c->dtype != B->vtype || a->dtype != B->vtype)
        return fail(ctx, SPL_ERR_DTYPE, "SpMV needs vals, c and a all F64 or all F32");
    Plan p;
    SPL_CHECK(resolve_spmv(ctx, B, sched, p));
    if (p.kind == SPL_NNZ || p.variant != 0)
        return fail(ctx, SPL_ERR_ARG, "a windowed SpMV runs the ROW or MERGE schedule (variant 0)");
    const int64_t n = B->dims[0];
    if (n == 0) return SPL_OK;
    if (!begin || !end) return fail(ctx, SPL_ERR_ARG, "NULL window bounds");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p.kind == SPL_ROW) {
        LeafTimer tm(ctx, SPL_OP_SPMV, s);
        SPL_HIP(spl::launch_spmv_row(B->vtype, p.lanes, n, begin, end, B->crd[1], B->vals,
                                     c->data, a->data, s),
                "windowed SpMV launch");
        tm.stop();
        return SPL_OK;
    }
    // Merge split over the windows: their lengths are scanned into virtual
    // positions on the device; the window total is at most nnz, so the tile
    // count is sized for nnz and the bounds read the total on the device.
    const Pieces q = pieces_for(p, n, B->nnz, spmv_chunk(p));
    const int64_t scan_tiles = spl::spadd3_scan_tiles(n);
    const size_t vpos_bytes = align_up(static_cast<size_t>(n + 1) * 4);
    const size_t scan_bytes = align_up(static_cast<size_t>(scan_tiles + 1) * 8);
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, nullptr, 0, vpos_bytes + scan_bytes + tiled_ws(q, 1, sizeof(double)),
                            &ws));
    char *wp = static_cast<char *>(ws);
    int32_t *vpos = reinterpret_cast<int32_t *>(wp);
    int64_t *tile_sum = reinterpret_cast<int64_t *>(wp + vpos_bytes);
    Carved cv = carve(wp + vpos_bytes + scan_bytes, q.count);
    SPL_HIP(spl::launch_window_offsets(n, begin, end, vpos, tile_sum, tile_sum + scan_tiles, s),
            "window offsets launch");
    SPL_HIP(spl::launch_tile_bounds(SPL_MERGE, n, vpos, /*total on the device*/ -1, q.size,
                                    cv.tiles, s),
            "tile bounds launch");
    LeafTimer tm(ctx, SPL_OP_SPMV, s);
    SPL_HIP(spl::launch_spmv_window_merge(B->vtype, p.items, n, vpos, begin, B->crd[1], B->vals,
                                          c->data, a->data, cv.tiles, q.stride,
                                          static_cast<double *>(cv.carry), s),
            "windowed SpMV launch");
    tm.stop();
    SPL_HIP(spl::launch_spmv_fixup(B->vtype, n, cv.tiles, q.stride,
                                   static_cast<double *>(cv.carry), a->data, s),
            "windowed SpMV fix-up launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spttv(spl_context *ctx, const spl_sparse *B, const spl_dense *c, spl_dense *A,
                     const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                     spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 3, true));
    SPL_CHECK(check_dense(ctx, c, "c", 1, B->dims[2], -1));
    SPL_CHECK(check_dense(ctx, A, "A", 1, B->nfibers, -1));
    if (B->vtype == SPL_BF16 || c->dtype != B->vtype || A->dtype != B->vtype)
        return fail(ctx, SPL_ERR_DTYPE, "SpTTV needs vals, c and A all F64 or all F32");
    const spl_sparse v = fiber_view(B);
    Plan p;
    SPL_CHECK(resolve_spmv(ctx, &v, sched, p));
    const bool pos64 = B->pos_type == SPL_I64;
    if (pos64 && (p.kind != SPL_MERGE || p.variant != 0))
        return fail(ctx, SPL_ERR_UNSUPPORTED, "int64 positions: MERGE schedule, variant 0 only");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t F = B->nfibers;
    if (F == 0) return SPL_OK;
    if (pos64) {
        // the fiber level's int64 positions: the SpMV flag leaf over fibers
        void *ws = nullptr;
        SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmv_ws(&v, p), &ws));
        const Pieces q = pieces_for(p, F, B->nnz, spmv_chunk(p));
        Carved cv = carve(ws, q.count, true);
        const int64_t *pos = reinterpret_cast<const int64_t *>(v.pos[1]);
        SPL_HIP(spl::launch_merge_bounds64(F, pos, B->nnz, q.size, cv.tiles, s),
                "tile bounds launch");
        LeafTimer tm(ctx, SPL_OP_SPTTV, s);
        SPL_HIP(spl::launch_spmv_flag64(B->vtype, p.items, F, pos, v.crd[1], B->vals, c->data,
                                        A->data, cv.tiles, q.stride,
                                        static_cast<double *>(cv.carry), s),
                "SpTTV tile launch");
        tm.stop();
        SPL_HIP(spl::launch_spmv_fixup(B->vtype, F, cv.tiles, q.stride,
                                       static_cast<double *>(cv.carry), A->data, s),
                "SpTTV fix-up launch");
        return SPL_OK;
    }
    if (p.kind == SPL_ROW) {
        LeafTimer tm(ctx, SPL_OP_SPTTV, s);
        SPL_HIP(spl::launch_spmv_row(B->vtype, p.lanes, F, v.pos[1], nullptr, v.crd[1], B->vals, c->data,
                                     A->data, s),
                "SpTTV row launch");
        tm.stop();
        return SPL_OK;
    }
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmv_ws(&v, p), &ws));
    const Pieces q = pieces_for(p, F, B->nnz, spmv_chunk(p));
    Carved cv = carve(ws, q.count);
    SPL_HIP(spl::launch_tile_bounds(p.kind, F, v.pos[1], B->nnz, q.size, cv.tiles, s),
            "tile bounds launch");
    LeafTimer tm(ctx, SPL_OP_SPTTV, s);
    SPL_HIP(spl::launch_spmv_tiles(B->vtype, p.items, F, v.pos[1], v.crd[1], B->vals, c->data,
                                   A->data, cv.tiles, q.stride, /*exact_chunks=*/p.kind == SPL_MERGE,
                                   p.variant, static_cast<double *>(cv.carry), s),
            "SpTTV tile launch");
    tm.stop();
    SPL_HIP(spl::launch_spmv_fixup(B->vtype, F, cv.tiles, q.stride,
                                   static_cast<double *>(cv.carry), A->data, s),
            "SpTTV fix-up launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mttkrp(spl_context *ctx, const spl_sparse *B, const spl_dense *C,
                      const spl_dense *D, spl_dense *A, const spl_schedule *sched,
                      void *workspace, size_t workspace_bytes, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 3, true));
    if (!C || !D) return fail(ctx, SPL_ERR_ARG, "dense factor is NULL");
    const bool pos64 = B->pos_type == SPL_I64;
    if (pos64 && dense_middle(B))
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "int64 positions: MTTKRP takes a Compressed middle level (CSF)");
    const int64_t R = C->ndim == 2 ? C->dims[1] : -1;
    SPL_CHECK(check_dense(ctx, C, "C", 2, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, D, "D", 2, B->dims[2], R));
    SPL_CHECK(check_dense(ctx, A, "A", 2, B->dims[0], R));
    const bool ok = A->dtype == SPL_F32 &&
                    ((B->vtype == SPL_F32 && C->dtype == SPL_F32 && D->dtype == SPL_F32) ||
                     (B->vtype == SPL_BF16 && C->dtype == SPL_BF16 && D->dtype == SPL_BF16));
    if (!ok)
        return fail(ctx, SPL_ERR_DTYPE,
                    "MTTKRP dtypes (vals, C, D, A) must be (F32,F32,F32,F32) or (BF16,BF16,BF16,F32)");
    Plan p;
    SPL_CHECK(resolve_mttkrp(ctx, R, sched, p));
    if (p.variant == 2 && B->vtype != SPL_BF16)
        return fail(ctx, SPL_ERR_ARG, "MTTKRP variant 2 (8-byte lanes) is for BF16 factors");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t I = B->dims[0];
    if (I == 0 || R == 0) return SPL_OK;
    // the workspace query took the largest size over the lane widths
    p.vec = mttkrp_vec(p, C, D, A);
    finish_mttkrp(p, pos64);
    if (p.variant == 3 && (B->vtype != SPL_F32 || p.items != 4))
        return fail(ctx, SPL_ERR_ARG,
                    "MTTKRP variant 3 (staged positions) is for F32 with items_per_lane 4");
    if (p.items == 3 && !(p.vec == 8 && p.col_tile == 32))
        return fail(ctx, SPL_ERR_ARG,
                    "MTTKRP items_per_lane 3 needs 8-column BF16 lanes (BF16 factors, variant 0, "
                    "col_tile 32, R and every ld multiples of 8, 16-byte aligned factors)");
    if (p.items == 5 && !(p.vec == 4 && p.col_tile == 32))
        return fail(ctx, SPL_ERR_ARG,
                    "MTTKRP items_per_lane 5 needs 4-column lanes at col_tile 32 (variant 0 or "
                    "2, R and every ld multiples of 4, aligned factors)");
    if (pos64 && (p.kind != SPL_MERGE || p.vec == 1))
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "int64 positions: MERGE schedule with vector lanes only (variant 0 or 2, "
                    "col_tile 32 or 64, items_per_lane 4 or 8, R and every ld multiples of 4)");
    if (p.items == 4 && p.vec == 1)
        return fail(ctx, SPL_ERR_ARG,
                    "MTTKRP items_per_lane 4 needs 4-column lanes (variant 0, col_tile 32 or 64, "
                    "R and every ld multiples of 4, 16-byte aligned factors)");
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes,
                            dense_middle_ws(B) + mttkrp_ws(B, R, p), &ws));
    char *wp = static_cast<char *>(ws);
    spl_sparse bv;
    SPL_CHECK(expand_middle(ctx, B, wp, bv, s));
    B = &bv;
    const Pieces q = mttkrp_pieces(B, p);
    Carved cv = carve(wp, q.count);
    const size_t fb = dtype_bytes(C->dtype);
    const bool buf = spl::mttkrp_buf(B->nnz, dtype_bytes(B->vtype), B->dims[1], C->ld, B->dims[2],
                                     D->ld, fb);
    if (pos64) {
        // slice ends are fiber indices (below 2^31): int32 tile bounds
        const int64_t *pos1 = reinterpret_cast<const int64_t *>(B->pos[1]);
        const int64_t *pos2 = reinterpret_cast<const int64_t *>(B->pos[2]);
        SPL_HIP(spl::launch_merge_bounds64_32(I, pos1, B->nfibers, q.size, cv.tiles, s),
                "tile bounds launch");
        LeafTimer tm(ctx, SPL_OP_MTTKRP, s);
        SPL_HIP(spl::launch_mttkrp_tiles64(B->vtype, buf, p.col_tile, p.items, p.vec, I, R, pos1,
                                           B->crd[1], pos2, B->crd[2], B->vals, C->data, C->ld,
                                           D->data, D->ld, static_cast<float *>(A->data), A->ld,
                                           cv.tiles, q.stride, static_cast<float *>(cv.carry), s),
                "MTTKRP tile launch");
        tm.stop();
        SPL_HIP(spl::launch_mttkrp_fixup(I, R, cv.tiles, q.stride, static_cast<float *>(cv.carry),
                                         static_cast<float *>(A->data), A->ld, s),
                "MTTKRP fix-up launch");
        return SPL_OK;
    }
    if (p.kind == SPL_NNZ)
        SPL_HIP(spl::launch_csf_nnz_bounds(I, B->pos[1], B->nfibers, B->pos[2], B->nnz, p.tile,
                                           cv.tiles, s),
                "CSF bounds launch");
    else
        SPL_HIP(spl::launch_tile_bounds(p.kind, I, B->pos[1], B->nfibers, q.size, cv.tiles, s),
                "tile bounds launch");
    LeafTimer tm(ctx, SPL_OP_MTTKRP, s);
    SPL_HIP(spl::launch_mttkrp_tiles(B->vtype, buf, p.variant == 3, p.col_tile, p.items, p.vec, I, R,
                                     B->pos[1], B->crd[1],
                                     B->pos[2], B->crd[2], B->vals, C->data, C->ld, D->data,
                                     D->ld, static_cast<float *>(A->data), A->ld, cv.tiles,
                                     q.stride, static_cast<float *>(cv.carry), s),
            "MTTKRP tile launch");
    tm.stop();
    SPL_HIP(spl::launch_mttkrp_fixup(I, R, cv.tiles, q.stride, static_cast<float *>(cv.carry),
                                     static_cast<float *>(A->data), A->ld, s),
            "MTTKRP fix-up launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_inner(spl_context *ctx, const spl_sparse *B, const spl_sparse *C, double *out,
                     const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                     spl_stream stream) {
    SPL_GUARD_BEGIN
    (void)sched;
    if (!ctx) return SPL_ERR_ARG;
    if (!B || !C || !out) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    const int order = B->order;
    if (order != 2 && order != 3) return fail(ctx, SPL_ERR_FORMAT, "order must be 2 or 3");
    SPL_CHECK(check_sparse(ctx, B, order));
    SPL_CHECK(check_sparse(ctx, C, order));
    if (!same_dims(B, C))
        return fail(ctx, SPL_ERR_SHAPE, "operands differ in shape");
    if (B->vtype != C->vtype || B->vtype == SPL_BF16)
        return fail(ctx, SPL_ERR_DTYPE, "inner product needs both F64 or both F32 values");
    // one pattern: the same arrays at every stored level (a Dense middle level
    // is the same for both once the shapes agree)
    bool shared = B->nnz == C->nnz && dense_middle(B) == dense_middle(C);
    for (int l = 1; l < order; ++l)
        if (!(l == 1 && dense_middle(B)))
            shared = shared && B->pos[l] == C->pos[l] && B->crd[l] == C->crd[l];
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    const size_t expand = shared ? 0 : dense_middle_ws(B) + dense_middle_ws(C);
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, expand + inner_ws(B), &ws));
    char *wp = static_cast<char *>(ws);
    spl_sparse bx, cx;
    if (!shared) {
        SPL_CHECK(expand_middle(ctx, B, wp, bx, s));
        SPL_CHECK(expand_middle(ctx, C, wp, cx, s));
        B = &bx;
        C = &cx;
    }
    ws = wp;
    LeafTimer tm(ctx, SPL_OP_INNER, s);
    if (shared) {
        // one pattern (the same pos/crd arrays): the aligned values' dot product
        SPL_HIP(spl::launch_inner(B->vtype, B->nnz, B->vals, C->vals, static_cast<double *>(ws),
                                  kInnerParts, out, s),
                "inner product launch");
    } else {
        const bool o3 = order == 3;
        SPL_HIP(spl::launch_inner_general(
                    B->vtype, order, B->dims[0], o3 ? B->nfibers : B->nnz, B->pos[1], B->crd[1],
                    o3 ? B->pos[2] : nullptr, o3 ? B->crd[2] : nullptr, B->vals, C->pos[1],
                    C->crd[1], o3 ? C->pos[2] : nullptr, o3 ? C->crd[2] : nullptr, C->vals,
                    B->nnz, C->nnz, o3 ? C->nfibers : C->nnz, ws, out, s),
                "inner product launch");
    }
    tm.stop();
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_sddmm(spl_context *ctx, const spl_sparse *B, const spl_dense *C,
                     const spl_dense *D, spl_dense *A, const spl_schedule *sched,
                     void *workspace, size_t workspace_bytes, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    if (!C || !D) return fail(ctx, SPL_ERR_ARG, "dense factor is NULL");
    const int64_t K = C->ndim == 2 ? C->dims[1] : -1;
    SPL_CHECK(check_dense(ctx, C, "C", 2, B->dims[0], -1));
    SPL_CHECK(check_dense(ctx, D, "D", 2, B->dims[1], K));
    SPL_CHECK(check_dense(ctx, A, "A", 1, B->nnz, -1));
    const bool ok = (B->vtype == SPL_F64 && C->dtype == SPL_F64 && D->dtype == SPL_F64 &&
                     A->dtype == SPL_F64) ||
                    (B->vtype == SPL_F32 && A->dtype == SPL_F32 && C->dtype == D->dtype &&
                     (C->dtype == SPL_F32 || C->dtype == SPL_BF16));
    if (!ok)
        return fail(ctx, SPL_ERR_DTYPE,
                    "SDDMM dtypes (vals, C, D, A) must be all F64, all F32 or (F32,BF16,BF16,F32)");
    Plan p;
    SPL_CHECK(resolve_sddmm(ctx, sched, p));
    const int variant = p.items;
    if (variant == 1) {
        if (C->dtype != SPL_BF16)
            return fail(ctx, SPL_ERR_UNSUPPORTED, "the matrix-core variant needs BF16 factors");
        if (K % 32 != 0 || C->ld % 8 != 0 || D->ld % 8 != 0 ||
            reinterpret_cast<uintptr_t>(C->data) % 16 != 0 ||
            reinterpret_cast<uintptr_t>(D->data) % 16 != 0)
            return fail(ctx, SPL_ERR_UNSUPPORTED,
                        "the matrix-core variant needs K % 32 == 0, ld % 8 == 0 and 16-byte "
                        "aligned factors");
    } else if (variant != 0) {
        return fail(ctx, SPL_ERR_ARG, "SDDMM variant must be 0 (VALU) or 1 (matrix cores)");
    }
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    if (n == 0 || B->nnz == 0) return SPL_OK;
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, sddmm_ws(B, p), &ws));
    const Pieces q = pieces_for(p, n, B->nnz, spl::sddmm_chunk());
    Carved cv = carve(ws, q.count);
    SPL_HIP(spl::launch_tile_bounds(p.kind, n, B->pos[1], B->nnz, q.size, cv.tiles, s),
            "tile bounds launch");
    // vector lanes for the VALU variant when K, the leading dimensions and
    // the factor pointers allow 16-byte accesses
    int vec_lanes = 0;
    if (variant == 0) {
        const int v = spl::sddmm_vec_width(C->dtype);
        if (K % v == 0 && C->ld % v == 0 && D->ld % v == 0 &&
            reinterpret_cast<uintptr_t>(C->data) % 16 == 0 &&
            reinterpret_cast<uintptr_t>(D->data) % 16 == 0)
            vec_lanes = K / v >= 32 ? 32 : K / v >= 16 ? 16 : 8;
    }
    LeafTimer tm(ctx, SPL_OP_SDDMM, s);
    SPL_HIP(spl::launch_sddmm(B->vtype, C->dtype, variant, vec_lanes, K, B->pos[1], B->crd[1], B->vals,
                              C->data, C->ld, D->data, D->ld, A->data, cv.tiles, q.stride, s),
            "SDDMM launch");
    tm.stop();
    return SPL_OK;
    SPL_GUARD_END
}

namespace {
// The numeric phase's default form (0 direct, 1 coordinates staged, 2
// coordinates and values staged, 3 by ranks).
constexpr int kSpadd3DefaultStage = 3;

// sched->variant (0..4) picks the numeric phase's form: 0 library default,
// 1..3 the merges (inputs read directly, coordinate runs staged in LDS,
// coordinates and values staged), 4 by ranks (coordinates staged, a lane per
// input entry).  The symbolic phase checks it and counts by merge always.
spl_status spadd3_variant(spl_context *ctx, const spl_schedule *sched, int *variant) {
    *variant = sched ? sched->variant : 0;
    if (*variant < 0 || *variant > 4) return fail(ctx, SPL_ERR_ARG, "SpAdd3 variant must be 0..4");
    return SPL_OK;
}

spl_status check_spadd3(spl_context *ctx, const spl_sparse *B, const spl_sparse *C,
                        const spl_sparse *D, const spl_schedule *sched) {
    SPL_CHECK(check_sparse(ctx, B, 2));
    SPL_CHECK(check_sparse(ctx, C, 2));
    SPL_CHECK(check_sparse(ctx, D, 2));
    if (!same_dims(B, C) || !same_dims(B, D))
        return fail(ctx, SPL_ERR_SHAPE, "SpAdd3 operands must have equal dimensions");
    if (sched && sched->kind != SPL_SCHED_DEFAULT && sched->kind != SPL_ROW)
        return fail(ctx, SPL_ERR_UNSUPPORTED,
                    "SpAdd3 on CSR supports only the row split (a non-zero split of a sum of "
                    "CSR operands does not align their positions)");
    return SPL_OK;
}
}  // namespace

spl_status spl_spadd3_symbolic(spl_context *ctx, const spl_sparse *B, const spl_sparse *C,
                               const spl_sparse *D, int32_t *A_pos, int64_t *nnz_out,
                               const spl_schedule *sched, void *workspace,
                               size_t workspace_bytes, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!A_pos || !nnz_out) return fail(ctx, SPL_ERR_ARG, "NULL output");
    SPL_CHECK(check_spadd3(ctx, B, C, D, sched));
    int variant = 0;
    SPL_CHECK(spadd3_variant(ctx, sched, &variant));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spadd3_ws(n), &ws));
    int64_t *tile_sum = static_cast<int64_t *>(ws);
    int64_t *total =
        reinterpret_cast<int64_t *>(static_cast<char *>(ws) +
                                    align_up(static_cast<size_t>(spl::spadd3_scan_tiles(n)) * 8));
    LeafTimer tm(ctx, SPL_OP_SPADD3, s);
    SPL_HIP(spl::launch_spadd3_symbolic(n, B->pos[1], B->crd[1], C->pos[1], C->crd[1], D->pos[1],
                                        D->crd[1], A_pos, tile_sum, total, s),
            "SpAdd3 symbolic launch");
    tm.stop();
    SPL_HIP(hipMemcpyAsync(ctx->readback, total, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync");
    SPL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    const int64_t host_total = ctx->readback[0];
    if (host_total > kIndexMax)
        return fail(ctx, SPL_ERR_SHAPE, "output nnz %lld exceeds int32 positions",
                    static_cast<long long>(host_total));
    *nnz_out = host_total;
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spadd3_numeric(spl_context *ctx, const spl_sparse *B, const spl_sparse *C,
                              const spl_sparse *D, const int32_t *A_pos, int32_t *A_crd,
                              void *A_vals, const spl_schedule *sched, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!A_pos) return fail(ctx, SPL_ERR_ARG, "NULL A_pos");
    SPL_CHECK(check_spadd3(ctx, B, C, D, sched));
    if (B->vtype != C->vtype || B->vtype != D->vtype || B->vtype == SPL_BF16)
        return fail(ctx, SPL_ERR_DTYPE, "SpAdd3 needs three F64 or three F32 operands");
    const int64_t n = B->dims[0];
    if (n > 0 && (B->nnz + C->nnz + D->nnz > 0) && (!A_crd || !A_vals))
        return fail(ctx, SPL_ERR_ARG, "NULL output arrays");
    int variant = 0;
    SPL_CHECK(spadd3_variant(ctx, sched, &variant));
    const int stage = variant == 0 ? kSpadd3DefaultStage : variant - 1;
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    LeafTimer tm(ctx, SPL_OP_SPADD3, s);
    SPL_HIP(spl::launch_spadd3_numeric(B->vtype, n, B->pos[1], B->crd[1], B->vals, C->pos[1],
                                       C->crd[1], C->vals, D->pos[1], D->crd[1], D->vals, A_pos,
                                       A_crd, A_vals, stage, s),
            "SpAdd3 numeric launch");
    tm.stop();
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_transpose_workspace_query(spl_context *ctx, const spl_sparse *B, size_t *bytes) {
    SPL_GUARD_BEGIN
    if (!ctx || !bytes) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    SPL_CHECK(check_sparse(ctx, B, 2));
    *bytes = spl::transpose_ws_bytes(B->nnz, B->dims[1]);
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_transpose(spl_context *ctx, const spl_sparse *B, int32_t *T_pos, int32_t *T_crd,
                         void *T_vals, void *workspace, size_t workspace_bytes,
                         spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    if (!T_pos || (B->nnz > 0 && (!T_crd || !T_vals)))
        return fail(ctx, SPL_ERR_ARG, "NULL output array");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes,
                            spl::transpose_ws_bytes(B->nnz, B->dims[1]), &ws));
    SPL_HIP(spl::launch_transpose(B->vtype, B->dims[0], B->dims[1], B->nnz, B->pos[1], B->crd[1],
                                  B->vals, T_pos, T_crd, T_vals, ws, s),
            "transpose launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_tin_workspace_query(spl_context *ctx, const char *tin, int nops,
                                   const spl_tin_operand *ops, const spl_tin_operand *out,
                                   size_t *bytes) {
    SPL_GUARD_BEGIN
    if (!ctx || !bytes) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    std::vector<spl::tin::Binding> b;
    spl::tin::Binding ob;
    spl::tin::Program prog;
    SPL_CHECK(tin_prepare(ctx, tin, nops, ops, out, b, ob, prog, nullptr));
    *bytes = spl::tin::workspace_bytes(prog, prog.out_kind == spl::tin::kOutCsr);
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_tin_source(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                          const spl_tin_operand *out, char *buf, size_t cap, size_t *len) {
    SPL_GUARD_BEGIN
    std::vector<spl::tin::Binding> b;
    spl::tin::Binding ob;
    spl::tin::Program prog;
    SPL_CHECK(tin_prepare(ctx, tin, nops, ops, out, b, ob, prog, nullptr));
    if (len) *len = prog.source.size();
    if (buf && cap) {
        const size_t n = std::min(cap - 1, prog.source.size());
        std::memcpy(buf, prog.source.data(), n);
        buf[n] = '\0';
    }
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_tin_symbolic(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                            const spl_tin_operand *out, int32_t *A_pos, int64_t *nnz_out,
                            void *workspace, size_t workspace_bytes, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!A_pos || !nnz_out) return fail(ctx, SPL_ERR_ARG, "NULL output");
    std::vector<spl::tin::Binding> b;
    spl::tin::Binding ob;
    spl::tin::Program prog, *cp = nullptr;
    SPL_CHECK(tin_prepare(ctx, tin, nops, ops, out, b, ob, prog, &cp));
    if (prog.out_kind != spl::tin::kOutCsr)
        return fail(ctx, SPL_ERR_ARG, "the symbolic phase is for sparse (CSR) outputs");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spl::tin::workspace_bytes(prog, true),
                            &ws));
    int64_t *tile_sum = static_cast<int64_t *>(ws);
    int64_t *total = reinterpret_cast<int64_t *>(
        static_cast<char *>(ws) + align_up(static_cast<size_t>(spl::spadd3_scan_tiles(prog.rows)) * 8));
    std::vector<unsigned long long> slots;
    spl::tin::fill_slots(prog, b, ob, A_pos, nullptr, nullptr, slots);
    SPL_HIP(tin_launch(cp->f_count, prog.rows, slots, s), "generated count launch");
    SPL_HIP(spl::launch_pos_scan(prog.rows, A_pos, tile_sum, total, s), "scan launch");
    SPL_HIP(hipMemcpyAsync(ctx->readback, total, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync");
    SPL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    const int64_t host_total = ctx->readback[0];
    if (host_total > kIndexMax)
        return fail(ctx, SPL_ERR_SHAPE, "output nnz %lld exceeds int32 positions",
                    static_cast<long long>(host_total));
    *nnz_out = host_total;
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_tin_eval(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                        const spl_tin_operand *out, void *workspace, size_t workspace_bytes,
                        spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    std::vector<spl::tin::Binding> b;
    spl::tin::Binding ob;
    spl::tin::Program prog, *cp = nullptr;
    SPL_CHECK(tin_prepare(ctx, tin, nops, ops, out, b, ob, prog, &cp));
    if (prog.out_kind == spl::tin::kOutCsr) {
        if (!out->sparse->pos[1] || (out->sparse->nnz > 0 && (!out->sparse->crd[1] ||
                                                               !out->sparse->vals)))
            return fail(ctx, SPL_ERR_ARG, "a sparse output needs pos (from spl_tin_symbolic), "
                                          "crd and vals");
    } else if (!out->dense->data) {
        return fail(ctx, SPL_ERR_ARG, "the output has no data");
    }
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spl::tin::workspace_bytes(prog, false),
                            &ws));
    char *wp = static_cast<char *>(ws);
    void *partials = nullptr, *scratch = nullptr;
    if (prog.out_kind == spl::tin::kOutScalar) {
        partials = wp;
        wp += align_up(static_cast<size_t>(prog.rows) * 8);
    }
    if (prog.scratch_rows) scratch = wp;
    std::vector<unsigned long long> slots;
    const int32_t *apos = prog.out_kind == spl::tin::kOutCsr ? out->sparse->pos[1] : nullptr;
    spl::tin::fill_slots(prog, b, ob, apos, partials, scratch, slots);
    hipFunction_t f = prog.out_kind == spl::tin::kOutCsr ? cp->f_fill : cp->f_eval;
    SPL_HIP(tin_launch(f, prog.rows, slots, s), "generated leaf launch");
    if (prog.out_kind == spl::tin::kOutScalar)
        SPL_HIP(spl::launch_inner_final(prog.rows, static_cast<const double *>(partials),
                                        static_cast<double *>(out->dense->data), s),
                "final reduction launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_features(spl_context *ctx, const spl_sparse *B, float *feat, void *workspace,
                        size_t workspace_bytes, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    if (!feat) return fail(ctx, SPL_ERR_ARG, "NULL feature output");
    SPL_CHECK(set_device(ctx));
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes,
                            static_cast<size_t>(spl::feature_ws_bytes()), &ws));
    SPL_HIP(spl::launch_features(B->dims[0], B->dims[1], B->pos[1], B->crd[1],
                                 static_cast<double *>(ws), feat,
                                 static_cast<hipStream_t>(stream)),
            "features launch");
    return SPL_OK;
    SPL_GUARD_END
}

int64_t spl_mlp_param_count(int K) {
    if (K < 1 || K > 256) return 0;
    return spl::mlp_param_count(K);
}

spl_status spl_mlp_forward(spl_context *ctx, int K, const float *params, const float *X,
                           const float *norm, int64_t batch, float *Y, float *act,
                           spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (K < 1 || K > 256) return fail(ctx, SPL_ERR_ARG, "K must be 1..256");
    if (batch < 0 || batch > (1LL << 31) - 1) return fail(ctx, SPL_ERR_ARG, "bad batch size");
    if (batch > 0 && (!params || !X || !Y)) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    SPL_CHECK(set_device(ctx));
    SPL_HIP(spl::launch_mlp_forward(K, params, X, norm, batch, Y, act,
                                    static_cast<hipStream_t>(stream)),
            "MLP forward launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mlp_backward(spl_context *ctx, int K, const float *params, int64_t batch,
                            const float *Y, const float *T, const float *act, float *grad,
                            float *loss, void *workspace, size_t workspace_bytes,
                            spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (K < 1 || K > 256) return fail(ctx, SPL_ERR_ARG, "K must be 1..256");
    if (batch < 1 || batch > (1LL << 31) - 1) return fail(ctx, SPL_ERR_ARG, "bad batch size");
    if (!params || !Y || !T || !act || !grad) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    SPL_CHECK(set_device(ctx));
    const size_t need = static_cast<size_t>((128 + K + 1) * batch) * sizeof(float);
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, need, &ws));
    float *dZ = static_cast<float *>(ws);
    float *loss_b = dZ + (128 + K) * batch;
    SPL_HIP(spl::launch_mlp_backward(K, params, batch, Y, T, act, dZ, loss_b, grad, loss,
                                     static_cast<hipStream_t>(stream)),
            "MLP backward launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_adam_step(spl_context *ctx, int64_t n, float *params, float *m, float *v,
                         const float *grad, float lr, float beta1, float beta2, float eps,
                         int step, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (n < 0 || step < 1) return fail(ctx, SPL_ERR_ARG, "bad size or step");
    if (n > 0 && (!params || !m || !v || !grad)) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    if (n == 0) return SPL_OK;
    SPL_CHECK(set_device(ctx));
    SPL_HIP(spl::launch_adam(n, params, m, v, grad, lr, beta1, beta2, eps, step,
                             static_cast<hipStream_t>(stream)),
            "Adam launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_autotune(spl_context *ctx, spl_op op, const spl_sparse *B, const spl_dense *X,
                        spl_dense *Y, const spl_schedule *candidates, int ncand, int reps,
                        spl_schedule *best, float *times_ms, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (sel_index(op) < 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "spl_autotune covers SpMV and SpMM");
    if (!best) return fail(ctx, SPL_ERR_ARG, "NULL best");
    if (reps < 1 || reps > 100) return fail(ctx, SPL_ERR_ARG, "reps must be 1..100");
    const spl_schedule *list = candidates;
    int n = ncand;
    if (!list) {
        if (ncand != 0) return fail(ctx, SPL_ERR_ARG, "NULL candidates with ncand != 0");
        const std::vector<spl_schedule> &d = default_candidates(op);
        list = d.data();
        n = static_cast<int>(d.size());
    }
    if (n < 1 || n > 4096) return fail(ctx, SPL_ERR_ARG, "ncand must be 1..4096");
    for (int i = 0; i < n; ++i)
        if (!concrete_kind(list[i].kind))
            return fail(ctx, SPL_ERR_ARG, "candidate %d: kind must be DEFAULT, ROW, NNZ or MERGE", i);
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    EventSet ev(2 * reps);
    for (hipEvent_t &e : ev.e) SPL_HIP(hipEventCreate(&e), "hipEventCreate");
    std::vector<float> med(n), t(reps);
    for (int i = 0; i < n; ++i) {
        auto call = [&]() {
            return op == SPL_OP_SPMV ? spl_spmv(ctx, B, X, Y, &list[i], nullptr, 0, stream)
                                     : spl_spmm(ctx, B, X, Y, &list[i], nullptr, 0, stream);
        };
        SPL_CHECK(call());  // untimed: first-touch effects and workspace growth
        for (int r = 0; r < reps; ++r) {
            SPL_HIP(hipEventRecord(ev.e[2 * r], s), "hipEventRecord");
            SPL_CHECK(call());
            SPL_HIP(hipEventRecord(ev.e[2 * r + 1], s), "hipEventRecord");
        }
        SPL_HIP(hipEventSynchronize(ev.e[2 * reps - 1]), "hipEventSynchronize");
        for (int r = 0; r < reps; ++r)
            SPL_HIP(hipEventElapsedTime(&t[r], ev.e[2 * r], ev.e[2 * r + 1]),
                    "hipEventElapsedTime");
        std::sort(t.begin(), t.end());
        med[i] = t[reps / 2];
    }
    const int k = static_cast<int>(std::min_element(med.begin(), med.end()) - med.begin());
    *best = list[k];
    if (times_ms) std::copy(med.begin(), med.end(), times_ms);
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mlp_load(spl_context *ctx, spl_op op, int K, const spl_schedule *candidates,
                        const float *params, const float *norm) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    const int i = sel_index(op);
    if (i < 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "schedule selectors cover SpMV and SpMM");
    if (K < 1 || K > 256) return fail(ctx, SPL_ERR_ARG, "K must be 1..256");
    if (!candidates || !params) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    for (int k = 0; k < K; ++k)
        if (!concrete_kind(candidates[k].kind))
            return fail(ctx, SPL_ERR_ARG, "candidate %d: kind must be DEFAULT, ROW, NNZ or MERGE", k);
    SPL_CHECK(set_device(ctx));
    SPL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");  // the old buffers may be in use
    spl_context::Selector &sl = ctx->sel[i];
    for (float **b : {&sl.params, &sl.norm, &sl.m, &sl.v, &sl.scratch}) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    sl = spl_context::Selector{};
    const int64_t np = spl::mlp_param_count(K);
    const size_t pb = static_cast<size_t>(np) * sizeof(float);
    for (auto [b, bytes] : {std::pair<float **, size_t>{&sl.params, pb}, {&sl.m, pb}, {&sl.v, pb},
                            {&sl.norm, 14 * sizeof(float)},
                            {&sl.scratch, static_cast<size_t>(8 + K) * sizeof(float)}}) {
        if (hipMalloc(reinterpret_cast<void **>(b), bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, SPL_ERR_NOMEM, "hipMalloc(%zu) for the selector failed", bytes);
        }
    }
    float ident[14];
    for (int j = 0; j < 7; ++j) {
        ident[j] = 0.0f;
        ident[7 + j] = 1.0f;
    }
    SPL_HIP(hipMemcpy(sl.params, params, pb, hipMemcpyHostToDevice), "hipMemcpy");
    SPL_HIP(hipMemcpy(sl.norm, norm ? norm : ident, sizeof ident, hipMemcpyHostToDevice),
            "hipMemcpy");
    SPL_HIP(hipMemset(sl.m, 0, pb), "hipMemset");
    SPL_HIP(hipMemset(sl.v, 0, pb), "hipMemset");
    sl.K = K;
    sl.nparams = np;
    sl.cands.assign(candidates, candidates + K);
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mlp_save(spl_context *ctx, spl_op op, int *K, int cap, spl_schedule *candidates,
                        float *params, float *norm) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    const int i = sel_index(op);
    if (i < 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "schedule selectors cover SpMV and SpMM");
    if (!K) return fail(ctx, SPL_ERR_ARG, "NULL K");
    const spl_context::Selector &sl = ctx->sel[i];
    if (sl.K == 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "no schedule selector installed");
    *K = sl.K;
    if (cap < sl.K) return SPL_OK;
    SPL_CHECK(set_device(ctx));
    SPL_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (candidates) std::copy(sl.cands.begin(), sl.cands.end(), candidates);
    if (params)
        SPL_HIP(hipMemcpy(params, sl.params, static_cast<size_t>(sl.nparams) * sizeof(float),
                          hipMemcpyDeviceToHost),
                "hipMemcpy");
    if (norm) SPL_HIP(hipMemcpy(norm, sl.norm, 14 * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mlp_predict(spl_context *ctx, spl_op op, const spl_sparse *B, spl_schedule *out,
                           spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    const int i = sel_index(op);
    if (i < 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "schedule selectors cover SpMV and SpMM");
    if (!out) return fail(ctx, SPL_ERR_ARG, "NULL output");
    const spl_context::Selector &sl = ctx->sel[i];
    if (sl.K == 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "no schedule selector installed (spl_mlp_load)");
    SPL_CHECK(check_sparse(ctx, B, 2));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *feat = sl.scratch, *Y = sl.scratch + 8;
    SPL_CHECK(spl_features(ctx, B, feat, nullptr, 0, stream));
    SPL_HIP(spl::launch_mlp_forward(sl.K, sl.params, feat, sl.norm, 1, Y, nullptr, s),
            "MLP forward launch");
    std::vector<float> y(sl.K);
    SPL_HIP(hipMemcpyAsync(y.data(), Y, y.size() * sizeof(float), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync");
    SPL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    const int k = static_cast<int>(std::min_element(y.begin(), y.end()) - y.begin());
    *out = sl.cands[k];
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_mlp_train_step(spl_context *ctx, spl_op op, const float *X, const float *T,
                              int64_t batch, float lr, float *loss, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    const int i = sel_index(op);
    if (i < 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "schedule selectors cover SpMV and SpMM");
    spl_context::Selector &sl = ctx->sel[i];
    if (sl.K == 0) return fail(ctx, SPL_ERR_UNSUPPORTED, "no schedule selector installed (spl_mlp_load)");
    if (batch < 1 || batch > (1LL << 24)) return fail(ctx, SPL_ERR_ARG, "batch must be 1..2^24");
    if (!X || !T) return fail(ctx, SPL_ERR_ARG, "NULL argument");
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int K = sl.K;
    // context workspace: activations, predictions, gradient, backward scratch
    const size_t n_act = static_cast<size_t>(128 + 7) * batch, n_y = static_cast<size_t>(K) * batch;
    const size_t n_dz = static_cast<size_t>(128 + K) * batch, n_lb = static_cast<size_t>(batch);
    const size_t need = (align_up(n_act * 4) + align_up(n_y * 4) + align_up(sl.nparams * 4) +
                         align_up(n_dz * 4) + align_up(n_lb * 4));
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, nullptr, 0, need, &ws));
    char *w = static_cast<char *>(ws);
    auto take = [&](size_t count) {
        float *p = reinterpret_cast<float *>(w);
        w += align_up(count * 4);
        return p;
    };
    float *act = take(n_act), *Y = take(n_y), *grad = take(sl.nparams), *dZ = take(n_dz),
          *loss_b = take(n_lb);
    SPL_HIP(spl::launch_mlp_forward(K, sl.params, X, sl.norm, batch, Y, act, s),
            "MLP forward launch");
    SPL_HIP(spl::launch_mlp_backward(K, sl.params, batch, Y, T, act, dZ, loss_b, grad, loss, s),
            "MLP backward launch");
    ++sl.step;
    SPL_HIP(spl::launch_adam(sl.nparams, sl.params, sl.m, sl.v, grad, lr, 0.9f, 0.999f, 1e-8f,
                             sl.step, s),
            "Adam launch");
    return SPL_OK;
    SPL_GUARD_END
}

}  // extern "C"
