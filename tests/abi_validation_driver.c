/* Host-only driver for the library's argument validation, built and run by
 * tests/test_abi_sanitized.py against a copy of the library whose host code is compiled
 * with AddressSanitizer and UndefinedBehaviorSanitizer.  Every call below must be
 * rejected on the host before any device work (no GPU is needed); the driver checks the
 * status codes and that each failure leaves an error text, and exits 0 only if all match.
 * Pointers are fake, 16-byte aligned addresses that validation never dereferences. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "accord.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
    const char* err = accord_last_error();
    if (got != want || (want != ACCORD_OK && (!err || !err[0]))) {
        printf("FAIL %s: status %d (want %d), error '%s'\n", what, got, want, err ? err : "");
        ++failures;
    }
}

int main(void) {
    float* F = (float*)(uintptr_t)(1u << 20);
    float* F2 = (float*)(uintptr_t)((1u << 20) + 256);
    double* D = (double*)(uintptr_t)((1u << 20) + 512);
    void* WS = (void*)(uintptr_t)(1u << 20);
    const size_t big = (size_t)1 << 40;

    accord_params prm;
    accord_default_params(&prm);
    accord_stats st;

    /* sizes and strings */
    if (accord_workspace_bytes(0, 10, NULL) != 0 || accord_workspace_bytes(10, 12, NULL) == 0) {
        printf("FAIL workspace sizes\n");
        ++failures;
    }
    for (int s = -1; s < 9; ++s)
        if (!accord_status_str(s)) ++failures;

    /* accord_fit */
    expect(accord_fit(NULL, 10, 12, F, &prm, &st, NULL, WS, big, NULL), 1, "fit X null");
    expect(accord_fit(F, 0, 12, F, &prm, &st, NULL, WS, big, NULL), 1, "fit n 0");
    expect(accord_fit(F, 10, (1 << 20) + 1, F, &prm, &st, NULL, WS, big, NULL), 1, "fit p big");
    expect(accord_fit(F, 10, 12, F, NULL, &st, NULL, WS, big, NULL), 1, "fit params null");
    expect(accord_fit(F, 10, 12, F, &prm, &st, NULL, NULL, big, NULL), 4, "fit ws null");
    expect(accord_fit(F, 10, 12, F, &prm, &st, NULL, (char*)WS + 16, big, NULL), 4, "fit ws align");
    expect(accord_fit(F, 10, 12, F, &prm, &st, NULL, WS, 10, NULL), 4, "fit ws small");
    {
        accord_params q = prm;
        q.lambda = NAN;
        expect(accord_fit(F, 10, 12, F, &q, &st, NULL, WS, big, NULL), 1, "fit lambda nan");
        q = prm;
        q.beta = 1.5;
        expect(accord_fit(F, 10, 12, F, &q, &st, NULL, WS, big, NULL), 1, "fit beta");
        q = prm;
        q.precision = 9;
        expect(accord_fit(F, 10, 12, F, &q, &st, NULL, WS, big, NULL), 5, "fit precision");
        q = prm;
        q.probe = 2;
        expect(accord_fit(F, 10, 12, F, &q, &st, NULL, WS, big, NULL), 1, "fit probe");
        q = prm;
        q.timing = -3;
        expect(accord_fit(F, 10, 12, F, &q, &st, NULL, WS, big, NULL), 1, "fit timing");
    }

    /* single steps */
    expect(accord_prox(F, F, 10, 0.0, 0.1, F2, D, WS, big, NULL), 1, "prox tau");
    expect(accord_prox(F, F, 10, 0.5, 0.1, F, D, WS, big, NULL), 1, "prox alias");
    expect(accord_prox(F, F, 10, 0.5, 0.1, F2, D, WS, 16, NULL), 4, "prox ws");
    expect(accord_prox_noalloc(F, F, 10, 0.0, 0.1, F2, D, NULL), 1, "prox_noalloc tau");
    expect(accord_prox_noalloc(F, F, 10, 0.5, -1.0, F2, D, NULL), 1, "prox_noalloc lambda");
    expect(accord_prox_noalloc(F, F, 10, 0.5, 0.1, F2, NULL, NULL), 1, "prox_noalloc red");
    expect(accord_grad(F, 0, 5, F, NULL, F, WS, big, NULL), 1, "grad n");
    expect(accord_grad(F, 5, 5, F, NULL, NULL, WS, big, NULL), 1, "grad G null");
    expect(accord_objective(F, 5, 5, F, -0.1, D, WS, big, NULL), 1, "objective lambda");
    expect(accord_objective(F, 5, 5, F, 0.1, D, WS, 8, NULL), 4, "objective ws");

    /* batched form */
    {
        int64_t n[2] = {10, 12};
        double lam[2] = {0.1, 0.2};
        accord_batch_stats bst[4];
        expect(accord_fit_batch(NULL, n, 2, 7, lam, 2, F, &prm, NULL, bst, NULL, WS, big, NULL), 1,
               "batch X null");
        expect(accord_fit_batch(F, n, 0, 7, lam, 2, F, &prm, NULL, bst, NULL, WS, big, NULL), 1,
               "batch nsub");
        double badlam[2] = {0.1, -1.0};
        expect(accord_fit_batch(F, n, 2, 7, badlam, 2, F, &prm, NULL, bst, NULL, WS, big, NULL),
               1, "batch lambda");
        expect(accord_fit_batch(F, n, 2, 7, lam, 2, F, &prm, NULL, bst, NULL, WS, 16, NULL), 4,
               "batch ws");
        if (accord_batch_workspace_bytes(n, 2, 0, 4, NULL) != 0) ++failures;
    }

    /* differentiation form */
    {
        double taus[2] = {0.5, -0.1};
        expect(accord_fbs_replay(F, 10, 5, F, taus, 2, 0.1, NULL, WS, big, NULL), 1, "replay tau");
        expect(accord_fbs_replay(F, 10, 5, F, NULL, 2, 0.1, NULL, WS, big, NULL), 1,
               "replay taus null");
        expect(accord_val_loss_grad(F, 10, 5, F, NULL, F2, WS, big, NULL), 1, "val out null");
        expect(accord_fbs_adjoint_step(F, 10, 5, F, 0.0, 0.1, F2, D, F2, WS, big, NULL), 1,
               "adjoint tau");
        if (accord_adjoint_workspace_bytes(0, 5) != 0) ++failures;
    }

    /* steps after the fit */
    {
        double out = 0.0;
        expect(accord_epbic(50, 15, 1.0, 0.0, 3, 0.0, &out), 1, "epbic gamma");
        expect(accord_epbic(50, 15, 1.0, 0.0, 15 * 14 + 1, 0.5, &out), 1, "epbic nnz");
        expect(accord_epbic(50, 15, 1.0, 0.0, 3, 0.5, &out), 0, "epbic ok");
        expect(accord_refit(F, 10, 12, NULL, 0.5, F, &prm, &st, NULL, WS, big, NULL), 1,
               "refit omega_hat");
        expect(accord_refit(F, 10, 12, F2, 1.5, F, &prm, &st, NULL, WS, big, NULL), 1,
               "refit phi");
        expect(accord_reparam(F, 10, NULL, NULL, NULL), 1, "reparam outputs");
        expect(accord_reparam(F, 10, F, NULL, NULL), 1, "reparam alias");
    }

    if (failures) {
        printf("%d validation check(s) failed\n", failures);
        return 1;
    }
    printf("validation OK\n");
    return 0;
}
