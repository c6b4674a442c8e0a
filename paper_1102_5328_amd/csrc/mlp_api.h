// Internal interface of the MLP cost-model kernels.
#pragma once
#include <stdint.h>

#define TQ_MLP_IN 5
#define TQ_MLP_H 64
#define TQ_MLP_NPARAM 8769

// Chooses the candidate (NB, IB) with the largest ensemble-mean predicted
// GFLOP/s for an M x N factorization in a batch of `batch`; *spread receives
// the ensemble's disagreement about that choice: the largest loss against
// its own best candidate that any model predicts for it.
// Synchronous (default stream). Returns 0 or a TILEQR_ERR_* code.
int tq_mlp_choose(const float *params_host, int nmodels, const float *fmean, const float *fstd,
                  float ymean, float ystd, const int *cand, int ncand, int64_t M, int64_t N,
                  int64_t batch, int *nb, int *ib, double *spread);
