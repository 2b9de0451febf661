// jit.hpp -- per-plan code generation of the fused pass kernels (see jit.cpp).
#pragma once

#include <string>
#include <vector>

#include "plan.hpp"

namespace qsv {

struct JitKernelRef {
    int which = 0;   // 0 forward pass, 1 backward pass
    int pass = 0;    // index into fwd_pass / bwd_pass
    int group = 0;   // compilation unit
    std::string name;
    std::string source;
};

struct JitModules {
    std::string arch;
    std::vector<JitKernelRef> refs;
    std::vector<std::vector<char>> codes;  // one code object per group
};

// HIP source of every pass kernel of a fused plan (one string), with the
// kernels split into compilation groups of at most max_ops_per_group ops.
std::string jit_source(const qsv_plan_t* p, std::vector<JitKernelRef>& refs, int max_ops_per_group);

// Generate and compile with hipRTC for `arch` ("" = the current device's).
// Fills `out` with code objects; on failure returns a QSV_ERR_* code and a
// message in `err`. No device state is touched unless arch is "".
int jit_compile(const qsv_plan_t* p, const std::string& arch, JitModules& out, std::string& err);

}  // namespace qsv
