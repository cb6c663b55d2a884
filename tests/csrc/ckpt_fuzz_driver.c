/* Test driver for the checkpoint reader built with host AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_checkpoint_fuzz.py): calls
 * llr_checkpoint_info on every file named on the command line, first for the
 * sizes and then for the interval edges, and prints one letter per file, A
 * (accepted) or R (refused).  A read past a buffer, an overflow or any
 * undefined operation in the parser aborts the run. */
#include <stdio.h>
#include <stdlib.h>

#include "../../include/llr.h"

int main(int argc, char **argv)
{
    for (int i = 1; i < argc; ++i) {
        int prec = -1, nl = -1, L[8], n[8];
        double dE[8];
        llr_params p;
        llr_status st = llr_checkpoint_info(argv[i], &prec, &nl, L, n, dE, NULL, &p);
        if (st != LLR_OK) {
            putchar('R');
            continue;
        }
        long tot = 0;
        for (int k = 0; k < nl; ++k) tot += n[k];
        double *E = (double *)malloc(sizeof(double) * (size_t)(tot > 0 ? tot : 1));
        st = llr_checkpoint_info(argv[i], &prec, &nl, L, n, dE, E, &p);
        free(E);
        putchar(st == LLR_OK ? 'A' : 'R');
    }
    putchar('\n');
    return 0;
}
