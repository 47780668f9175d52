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

#include "internal.hpp"
#include "spleaf.h"

struct spl_context {
    int device = 0;
    std::string err;
    void *ws = nullptr;   // context-owned workspace (used when the caller gives none)
    size_t ws_bytes = 0;
    int64_t *flags = nullptr;  // 2 x int64 device scratch for spl_validate
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

spl_status check_sparse(spl_context *ctx, const spl_sparse *B, int order) {
    if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
    if (B->order != order)
        return fail(ctx, SPL_ERR_FORMAT, "expected an order-%d sparse operand, got order %d", order,
                    B->order);
    if (B->level[0] != SPL_DENSE)
        return fail(ctx, SPL_ERR_FORMAT, "level 0 must be Dense");
    for (int l = 1; l < order; ++l)
        if (B->level[l] != SPL_COMPRESSED)
            return fail(ctx, SPL_ERR_FORMAT, "level %d must be Compressed", l);
    if (!valid_dtype(B->vtype)) return fail(ctx, SPL_ERR_DTYPE, "unknown value dtype %d", B->vtype);
    for (int l = 0; l < order; ++l)
        if (B->dims[l] < 0 || B->dims[l] > kIndexMax)
            return fail(ctx, SPL_ERR_SHAPE, "dimension %d = %lld out of range", l,
                        static_cast<long long>(B->dims[l]));
    if (B->nnz < 0 || B->nnz > kIndexMax)
        return fail(ctx, SPL_ERR_SHAPE, "nnz = %lld out of range", static_cast<long long>(B->nnz));
    if (order == 3 && (B->nfibers < 0 || B->nfibers > kIndexMax))
        return fail(ctx, SPL_ERR_SHAPE, "nfibers = %lld out of range",
                    static_cast<long long>(B->nfibers));
    for (int l = 1; l < order; ++l) {
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
};

int lanes_for_mean(double mean) {
    int L = 1;
    while (L < 64 && L < mean) L <<= 1;
    return L;
}

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
    p.tile = s->tile ? s->tile : (p.kind == SPL_ROW ? 256 / p.lanes : 256 * p.items);
    if (p.tile < 1) return fail(ctx, SPL_ERR_ARG, "tile must be positive");
    return SPL_OK;
}

spl_status resolve_spmm(spl_context *ctx, const spl_sparse *B, int64_t N, const spl_schedule *s,
                        Plan &p) {
    (void)B;
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
    return SPL_OK;
}

// Workspace of a tiled leaf: tile bounds then per-tile carries.
size_t tiled_bytes(int64_t ntiles, int64_t carry_elems_per_tile, size_t carry_elem) {
    return 2 * align_up(static_cast<size_t>(ntiles + 1) * 4) +
           align_up(static_cast<size_t>(ntiles) * carry_elems_per_tile * carry_elem);
}

struct Carved {
    Tiles tiles;
    void *carry;
};

Carved carve(void *ws, int64_t ntiles) {
    char *b = static_cast<char *>(ws);
    Carved c;
    c.tiles.ntiles = ntiles;
    c.tiles.row = reinterpret_cast<int32_t *>(b);
    b += align_up(static_cast<size_t>(ntiles + 1) * 4);
    c.tiles.pos = reinterpret_cast<int32_t *>(b);
    b += align_up(static_cast<size_t>(ntiles + 1) * 4);
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

size_t spmv_ws(const spl_sparse *B, const Plan &p) {
    if (p.kind == SPL_ROW) return 0;
    const int64_t nt = spl::tile_count(p.kind, B->dims[0], B->nnz, p.tile);
    return tiled_bytes(nt, 1, sizeof(double));
}

size_t spmm_ws(const spl_sparse *B, int64_t N, const Plan &p) {
    if (p.kind == SPL_ROW) return 0;
    const int64_t nt = spl::tile_count(p.kind, B->dims[0], B->nnz, p.tile);
    return tiled_bytes(nt, N, B->vtype == SPL_F64 ? 8 : 4);
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
        hipMalloc(reinterpret_cast<void **>(&ctx->flags), 2 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return SPL_ERR_HIP;
    }
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
    delete ctx;
    return SPL_OK;
    SPL_GUARD_END
}

const char *spl_last_error(const spl_context *ctx) { return ctx ? ctx->err.c_str() : ""; }

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
        SPL_CHECK(check_sparse(ctx, B, 2));
        SPL_CHECK(resolve_spmv(ctx, B, sched, p));
        *bytes = spmv_ws(B, p);
        return SPL_OK;
    case SPL_OP_SPMM:
        SPL_CHECK(check_sparse(ctx, B, 2));
        SPL_CHECK(resolve_spmm(ctx, B, ncols, sched, p));
        *bytes = spmm_ws(B, ncols, p);
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

spl_status spl_validate(spl_context *ctx, const spl_sparse *B, spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    if (!B) return fail(ctx, SPL_ERR_ARG, "sparse operand is NULL");
    SPL_CHECK(check_sparse(ctx, B, B->order == 3 ? 3 : 2));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = 1; l < B->order; ++l) {
        const int64_t parents = l == 1 ? B->dims[0] : B->nfibers;
        const int64_t children = l == B->order - 1 ? B->nnz : B->nfibers;
        const int64_t extent = B->dims[l];
        const int64_t init[2] = {0, -1};
        SPL_HIP(hipMemcpyAsync(ctx->flags, init, sizeof init, hipMemcpyHostToDevice, s),
                "hipMemcpyAsync");
        SPL_HIP(spl::launch_validate_level(parents, B->pos[l], B->crd[l], children, extent,
                                           ctx->flags, s),
                "validate launch");
        int64_t res[2];
        SPL_HIP(hipMemcpyAsync(res, ctx->flags, sizeof res, hipMemcpyDeviceToHost, s),
                "hipMemcpyAsync");
        SPL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
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

spl_status spl_spmv(spl_context *ctx, const spl_sparse *B, const spl_dense *c, spl_dense *a,
                    const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                    spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    SPL_CHECK(check_dense(ctx, c, "c", 1, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, a, "a", 1, B->dims[0], -1));
    if (B->vtype == SPL_BF16 || c->dtype != B->vtype || a->dtype != B->vtype)
        return fail(ctx, SPL_ERR_DTYPE, "SpMV needs vals, c and a all F64 or all F32");
    Plan p;
    SPL_CHECK(resolve_spmv(ctx, B, sched, p));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    if (n == 0) return SPL_OK;
    if (p.kind == SPL_ROW) {
        SPL_HIP(spl::launch_spmv_row(B->vtype, p.lanes, n, B->pos[1], B->crd[1], B->vals, c->data,
                                     a->data, s),
                "SpMV row launch");
        return SPL_OK;
    }
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmv_ws(B, p), &ws));
    const int64_t nt = spl::tile_count(p.kind, n, B->nnz, p.tile);
    Carved cv = carve(ws, nt);
    SPL_HIP(spl::launch_tile_bounds(p.kind, n, B->pos[1], B->nnz, p.tile, cv.tiles, s),
            "tile bounds launch");
    SPL_HIP(spl::launch_spmv_tiles(B->vtype, p.items, n, B->pos[1], B->crd[1], B->vals, c->data,
                                   a->data, cv.tiles, static_cast<double *>(cv.carry), s),
            "SpMV tile launch");
    return SPL_OK;
    SPL_GUARD_END
}

spl_status spl_spmm(spl_context *ctx, const spl_sparse *B, const spl_dense *C, spl_dense *A,
                    const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                    spl_stream stream) {
    SPL_GUARD_BEGIN
    if (!ctx) return SPL_ERR_ARG;
    SPL_CHECK(check_sparse(ctx, B, 2));
    if (!C) return fail(ctx, SPL_ERR_ARG, "dense operand C is NULL");
    const int64_t N = C->ndim == 2 ? C->dims[1] : -1;
    SPL_CHECK(check_dense(ctx, C, "C", 2, B->dims[1], -1));
    SPL_CHECK(check_dense(ctx, A, "A", 2, B->dims[0], N));
    const bool ok = (B->vtype == SPL_F64 && C->dtype == SPL_F64 && A->dtype == SPL_F64) ||
                    (B->vtype == SPL_F32 && C->dtype == SPL_F32 && A->dtype == SPL_F32) ||
                    (B->vtype == SPL_BF16 && C->dtype == SPL_BF16 && A->dtype == SPL_F32);
    if (!ok)
        return fail(ctx, SPL_ERR_DTYPE,
                    "SpMM dtypes (vals, C, A) must be (F64,F64,F64), (F32,F32,F32) or (BF16,BF16,F32)");
    Plan p;
    SPL_CHECK(resolve_spmm(ctx, B, N, sched, p));
    SPL_CHECK(set_device(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = B->dims[0];
    if (n == 0 || N == 0) return SPL_OK;
    if (p.kind == SPL_ROW) {
        SPL_HIP(spl::launch_spmm_row(B->vtype, A->dtype, p.col_tile, n, N, B->pos[1], B->crd[1],
                                     B->vals, C->data, C->ld, A->data, A->ld, s),
                "SpMM row launch");
        return SPL_OK;
    }
    void *ws = nullptr;
    SPL_CHECK(get_workspace(ctx, workspace, workspace_bytes, spmm_ws(B, N, p), &ws));
    const int64_t nt = spl::tile_count(p.kind, n, B->nnz, p.tile);
    Carved cv = carve(ws, nt);
    SPL_HIP(spl::launch_tile_bounds(p.kind, n, B->pos[1], B->nnz, p.tile, cv.tiles, s),
            "tile bounds launch");
    SPL_HIP(spl::launch_spmm_tiles(B->vtype, A->dtype, p.col_tile, p.items, n, N, B->pos[1],
                                   B->crd[1], B->vals, C->data, C->ld, A->data, A->ld, cv.tiles,
                                   cv.carry, s),
            "SpMM tile launch");
    return SPL_OK;
    SPL_GUARD_END
}

}  // extern "C"
