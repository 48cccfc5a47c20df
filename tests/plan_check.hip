// Host-only check that the planning pass of every entry point sizes the
// workspace its executing pass uses.  All library sources are built into one
// translation unit with every kernel launch recorded (launch_op) or dropped
// (direct launches and the few HIP calls the executing pass makes), so the
// host logic of both passes runs on a machine without a GPU, over fake device
// addresses that are never dereferenced.  Prints one line per case and
// exits nonzero if any executing pass takes more workspace than its plan.
#include <hip/hip_runtime.h>
#include "common.h"
#undef RSVD_LAUNCH_CHECK
#define RSVD_LAUNCH_CHECK() do {} while (0)
static hipError_t plan_check_ok() { return hipSuccess; }
#define hipFuncSetAttribute(...) plan_check_ok()
#define hipMemcpyAsync(...) plan_check_ok()
#define hipPeekAtLastError() plan_check_ok()
#undef hipLaunchKernelGGL
#define hipLaunchKernelGGL(...) ((void)0)
#include "philox.hip"
#include "views.hip"
#include "views_lp.hip"
#include "orth.hip"
#include "small.hip"
#include "grad.hip"
#include "srft.hip"
#include "rsvd_api.hip"
#include <stdio.h>
#include <vector>

struct CountLaunches : LaunchRecorder {
    size_t n = 0;
    void add(const void*, const void*, const void*, size_t, dim3, unsigned, size_t) override { ++n; }
};

struct Case {
    const char* what;
    int kind;              // 0: rsvd_* entry (algo), 1: normal matrix, 2: gradient
    int algo;
    rsvd_dtype dt;
    int64_t m, n;
    int trans, k, p, v;
    rsvd_opts o;
};

static const char* kFakeA = (const char*)0x7f0000000000ull;
static char* const kFakeWs = (char*)0x7d0000000000ull;

static bool run_case(const Case& c) {
    rsvd_mat A{};
    A.dtype = c.dt;
    A.m = c.m;
    A.n = c.n;
    A.trans = c.trans;
    A.ld = c.trans ? (c.m + 7) / 8 * 8 : (c.n + 7) / 8 * 8;
    A.data = kFakeA;
    A.row_scale = c.dt == RSVD_FP8_E4M3 ? (const float*)0x7e8000000000ull : nullptr;
    rsvd_status perr = RSVD_OK;
    size_t need = 0;
    if (c.kind == 0) need = plan_bytes(&A, c.k, c.p, c.v, c.algo, c.o, &perr);
    else if (c.kind == 1) need = normal_plan_bytes(&A, c.k, c.p, c.v, c.algo, c.o, &perr);
    else need = grad_plan_bytes(&A, c.k, c.p, c.v, c.o, 1, &perr);
    CountLaunches rec;
    launch_recorder() = &rec;
    Ctx ctx{false, nullptr, Arena{kFakeWs}};
    ctx.status = (uint32_t*)kFakeWs;
    ctx.flags = (int*)(kFakeWs + 32);
    ctx.f32_mode = c.o.f32_mode;
    rsvd_out out{(void*)0x7c0000000000ull, (double*)0x7c1000000000ull, (void*)0x7c2000000000ull};
    rsvd_status e;
    if (c.kind == 0) {
        e = dispatch(ctx, c.algo, make_mat(&A), c.k, c.p, c.v, c.o, &out);
    } else if (c.kind == 1) {
        e = alg_normal(ctx, make_mat(&A), c.k, c.p, c.v, c.algo, c.o, (void*)0x7c3000000000ull,
                       (double*)0x7c4000000000ull);
    } else {
        double E = 0.0;
        e = alg_row_sweep_grad(ctx, make_mat(&A), c.k, c.p, c.v, c.o, &out, &E, (const double*)0x7c5000000000ull,
                               1.0, (void*)0x7c6000000000ull, c.n);
    }
    launch_recorder() = nullptr;
    const bool ok = perr == RSVD_OK && e == RSVD_OK && ctx.ar.off <= need;
    printf("%-44s %s %6ldx%-6ld t%d k%-3d p%-3d v%d: plan %10zu used %10zu launches %4zu  %s\n", c.what,
           c.dt == RSVD_F64 ? "f64" : c.dt == RSVD_F32 ? "f32" : c.dt == RSVD_BF16 ? "bf16" : "fp8", (long)c.m,
           (long)c.n, c.trans, c.k, c.p, c.v, need, ctx.ar.off, rec.n,
           ok ? "ok" : (perr != RSVD_OK || e != RSVD_OK ? "ERROR" : "OVERFLOW"));
    if (perr != RSVD_OK || e != RSVD_OK) printf("    status: plan %d, run %d\n", perr, e);
    return ok;
}

int main() {
    std::vector<Case> cases;
    auto base = [](const char* what, int kind, int algo, rsvd_dtype dt, int64_t m, int64_t n, int trans, int k, int p,
                   int v) {
        Case c{what, kind, algo, dt, m, n, trans, k, p, v, {}};
        rsvd_default_opts(&c.o);
        return c;
    };
    const int64_t shapes[][2] = {{700, 333}, {2000, 1000}, {333, 700}, {1200, 700}, {5000, 257}};
    for (rsvd_dtype dt : {RSVD_F64, RSVD_F32}) {
        for (auto& sh : shapes) {
            for (int trans : {0, 1}) {
                for (int v : {2, 3, 6}) cases.push_back(base("subspace", 0, ALG_SUB, dt, sh[0], sh[1], trans, 9, 5, v));
                cases.push_back(base("one view, Tropp, l_c = l_1", 0, ALG_ONE, dt, sh[0], sh[1], trans, 9, 5, 1));
                Case c = base("one view, Tropp, l_c = 2", 0, ALG_ONE, dt, sh[0], sh[1], trans, 9, 5, 1);
                c.o.lc_rule = RSVD_LC_FIXED;
                c.o.lc = 2;
                cases.push_back(c);
                c.what = "one view, Woolfe, minimum variance";
                c.o.one_view_method = RSVD_ONE_VIEW_WOOLFE;
                c.o.lc_rule = RSVD_LC_MINVAR;
                cases.push_back(c);
                c = base("one view, fixed ratio, s_w = 40", 0, ALG_ONE, dt, sh[0], sh[1], trans, 9, 5, 1);
                c.o.lc_rule = RSVD_LC_RATIO;
                c.o.lc_alpha = 0.5;
                c.o.psi_rows = 40;
                cases.push_back(c);
                c = base("one view, 256-row panels", 0, ALG_ONE, dt, sh[0], sh[1], trans, 9, 5, 1);
                c.o.block_rows = 256;
                cases.push_back(c);
                c = base("extended one view, Gaussian core", 0, ALG_ONE, dt, sh[0], sh[1], trans, 9, 5, 1);
                c.o.core_rows = 40;
                cases.push_back(c);
                c.what = "extended one view, SRFT core";
                c.o.core_kind = RSVD_CORE_SRFT;
                cases.push_back(c);
                for (int mode : {RSVD_KRYLOV_ALTERNATING, RSVD_KRYLOV_ROW_SWEEP, RSVD_KRYLOV_COL_SWEEP}) {
                    c = base("block Krylov", 0, ALG_KRY, dt, sh[0], sh[1], trans, 9, 5, 3);
                    c.o.krylov_mode = mode;
                    c.o.block_rows = 256;
                    cases.push_back(c);
                }
                for (int method : {NORMAL_NYSTROM, NORMAL_PINCHED, NORMAL_SUBSPACE})
                    cases.push_back(base("normal matrix", 1, method, dt, sh[0], sh[1], trans, 9, 5, 3));
            }
            Case g = base("row-sweep gradient", 2, 0, dt, sh[0], sh[1], 0, 9, 5, 3);
            g.o.krylov_mode = RSVD_KRYLOV_ROW_SWEEP;
            g.o.block_rows = 256;
            cases.push_back(g);
        }
    }
    for (rsvd_dtype dt : {RSVD_BF16, RSVD_FP8_E4M3}) {
        for (int v : {2, 3}) {
            Case c = base("low precision + refinement view", 0, ALG_SUB, dt, 4096, 1536, 0, 60, 20, v);
            c.o.refine = 1;
            cases.push_back(c);
        }
    }
    int bad = 0;
    for (const Case& c : cases) bad += !run_case(c);
    printf("%zu cases, %d failed\n", cases.size(), bad);
    return bad ? 1 : 0;
}
