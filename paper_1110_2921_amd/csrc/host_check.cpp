// Driver of the library's host layer for a build with AddressSanitizer: the
// context-free entry points (offset table, M2L lists, operator generation for
// every degree) and the argument checks of every entry point on a null
// context, none of which touches a device.  Prints OK when every call
// returned what its declaration promises.
#include "../../include/vmfmm.h"

#include <cstdio>
#include <vector>

int main() {
    int failures = 0;
    auto expect = [&](bool ok, const char *what) {
        if (!ok) {
            std::printf("FAIL %s\n", what);
            ++failures;
        }
    };
    int8_t offs[316 * 3];
    int count = 0;
    expect(vm_debug_offsets(offs, &count) == VM_OK && count == 316, "vm_debug_offsets");
    int32_t src[189];
    int8_t d[189 * 3], img[189 * 3];
    for (int level = 0; level <= 4; ++level)
        for (int periodic = 0; periodic <= 1; ++periodic)
            for (int32_t key = 0; key < (1 << (3 * level)); key += 1 + (level >= 3 ? 37 : 0)) {
                const vm_status st = vm_debug_list(level, periodic, key, src, d, img, &count);
                if (level >= 1 && (periodic || level >= 2))
                    expect(st == VM_OK && count >= 0 && count <= 189, "vm_debug_list");
                else
                    expect(st == VM_EINVAL, "vm_debug_list level range");
            }
    expect(vm_debug_list(2, 0, 1 << 6, src, d, img, &count) == VM_EINVAL, "vm_debug_list key range");
    for (int p = 1; p <= VM_MAX_P; ++p) {
        const int C = (p + 1) * (p + 1);
        std::vector<double> m(size_t(C) * C);
        expect(vm_debug_operator(0, p, p % 316, m.data()) == VM_OK, "M2L operator");
        expect(vm_debug_operator(1, p, p % 8, m.data()) == VM_OK, "M2M operator");
        expect(vm_debug_operator(2, p, p % 8, m.data()) == VM_OK, "L2L operator");
        if (p <= 8) expect(vm_debug_operator(3, p, 1 + p % 3, m.data()) == VM_OK, "lattice operator");
    }
    expect(vm_debug_operator(0, VM_MAX_P + 1, 0, nullptr) == VM_EINVAL, "operator degree range");
    // every entry point rejects a null context before anything else
    vm_opts o{};
    double buf[9] = {0};
    int32_t ibuf[8] = {0};
    int64_t rows = 0;
    int lvl = 0;
    expect(vm_fmm_eval(nullptr, 1, buf, buf, 1.0, 4, 2, &o, buf, buf, buf) == VM_EINVAL, "vm_fmm_eval");
    expect(vm_fmm_eval_at(nullptr, 1, buf, buf, 1, buf, 1.0, 4, 2, &o, buf, buf) == VM_EINVAL, "vm_fmm_eval_at");
    expect(vm_fmm_eval_adaptive(nullptr, 1, buf, buf, 1.0, 4, 8, 2, &o, buf, buf, buf) == VM_EINVAL,
           "vm_fmm_eval_adaptive");
    expect(vm_fmm_adjoint(nullptr, 1, buf, buf, 1.0, 4, 2, &o, buf, buf, buf) == VM_EINVAL, "vm_fmm_adjoint");
    expect(vm_rk2_step(nullptr, 1, buf, buf, 1.0, 4, 2, &o, 0.1, buf, buf) == VM_EINVAL, "vm_rk2_step");
    expect(vm_diagnostics(nullptr, 1, buf, buf, buf, 1.0, buf) == VM_EINVAL, "vm_diagnostics");
    expect(vm_diagnostics_noalloc(nullptr, 1, buf, buf, buf, 1.0, buf) == VM_EINVAL, "vm_diagnostics_noalloc");
    expect(vm_gauss_sum(nullptr, 1, buf, buf, 1.0, 2, &o, buf) == VM_EINVAL, "vm_gauss_sum");
    expect(vm_tune_level(nullptr, 1, buf, buf, 1.0, 4, &o, 4.0, 1, &lvl, buf) == VM_EINVAL, "vm_tune_level");
    expect(vm_tune_ncrit(nullptr, 1, buf, buf, 1.0, 4, 2, &o, 1, &lvl, buf) == VM_EINVAL, "vm_tune_ncrit");
    expect(vm_debug_adaptive(nullptr, 0, ibuf, &rows) == VM_EINVAL, "vm_debug_adaptive");
    expect(vm_set_timing(nullptr, 1) == VM_EINVAL, "vm_set_timing");
    expect(vm_last_error(nullptr) != nullptr, "vm_last_error");
    vm_destroy(nullptr);
    std::printf(failures ? "FAILED %d\n" : "OK\n", failures);
    return failures ? 1 : 0;
}
