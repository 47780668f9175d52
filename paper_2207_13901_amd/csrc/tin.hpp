// Index-notation front-end and leaf generator (host side).
//
// A statement of tensor index notation (Sec. II-A) over Dense/Compressed
// operands is parsed, given a concordant loop order (each sparse operand's
// levels iterated outer to inner, Sec. IV-C), and lowered to a loop nest in
// which every index variable is either a coordinate-value loop (a dense
// range) or a merge over the positions of the Compressed levels that index
// it (coordinate-position loops, co-iterated: intersection for products,
// union for sums; Sec. IV-C).  The nest is emitted as HIP source, compiled
// at run time for gfx950 and launched one thread per coordinate of the
// outermost index.  Outputs: a dense tensor (every entry written), a scalar,
// or a CSR matrix assembled in two phases (count, scan, fill; Sec. V-B).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "spleaf.h"

namespace spl {
namespace tin {

enum OutKind { kOutDense = 0, kOutScalar = 1, kOutCsr = 2 };

// One operand of a statement as the caller binds it: exactly one of
// sparse / dense is set.
struct Binding {
    std::string name;
    const spl_sparse *sparse = nullptr;
    const spl_dense *dense = nullptr;
};

// One kernel-argument slot: what the host writes into it.
struct Slot {
    enum Kind { kRows, kExtent, kPos, kCrd, kVals, kDenseData, kDenseLd, kLevelDim,
                kOutData, kOutLd, kOutPos, kOutCrd, kOutVals, kPartials, kScratch } kind;
    int operand = -1;  // index into the bindings (right side), -1 for the output
    int level = 0;     // sparse level, or the variable for kExtent
};

// A planned and generated statement for one set of operand formats.
struct Program {
    std::string key;
    std::string source;
    int out_kind = kOutDense;
    int vtype = SPL_F64;          // value type of every operand and the output
    int64_t rows = 0;             // extent of the outermost index (threads)
    int64_t out_cols = 1;         // dense output: entries per outermost coordinate
    std::vector<int64_t> extents; // per index variable, from this call's operands
    bool scratch_rows = false;    // dense F32 output accumulated in an F64 scratch
    std::vector<Slot> slots;
    hipModule_t module = nullptr;
    hipFunction_t f_eval = nullptr, f_count = nullptr, f_fill = nullptr;
    ~Program();
};

// Parse `stmt`, check it against the bindings and plan the loop nest.
// `out` is the left side's binding (its sparse/dense pointers may hold
// placeholders: only formats, dtypes and dimensions are read here).
// Returns SPL_OK or a status with the reason in `err`.
spl_status plan(const char *stmt, const std::vector<Binding> &ops, const Binding &out,
                Program &prog, std::string &err);

// Compile prog.source with hiprtc for gfx950 and load it on the current
// device.
spl_status compile(Program &prog, std::string &err);

// Kernel-argument slots for one call (64-bit each, in the order of
// prog.slots).  `out` as bound for this call; `partials` and `scratch` are
// device workspace pointers (may be null when unused).
void fill_slots(const Program &prog, const std::vector<Binding> &ops, const Binding &out,
                const int32_t *out_pos, void *partials, void *scratch,
                std::vector<unsigned long long> &slots);

// Workspace bytes a call of `prog` needs (partials, F64 row scratch, scan
// space for the symbolic phase), at 256-byte granularity.
size_t workspace_bytes(const Program &prog, bool symbolic);

}  // namespace tin
}  // namespace spl
