// Batched small factorizations (placeholder entry points; see skltlt.h).
#include "../../include/skltlt.h"
#include "common.h"

extern "C" int skltlt_batched_max_n(void) { return 0; }

extern "C" int skltlt_batched_workspace_size(int batch, size_t *bytes)
{
    if (batch < 0 || !bytes)
        return SKLTLT_EINVAL;
    *bytes = 0;
    return SKLTLT_ENOTSUP;
}

extern "C" int skltlt_batched(int batch, const int *n, double *const *A, const int *lda,
                              double *const *t, int *const *ipiv, double *log_abs_pf, int *sign,
                              int *info, int max_n, int block_size, int precision, void *work,
                              size_t work_bytes, void *stream)
{
    (void)batch; (void)n; (void)A; (void)lda; (void)t; (void)ipiv; (void)log_abs_pf;
    (void)sign; (void)info; (void)max_n; (void)block_size; (void)precision; (void)work;
    (void)work_bytes; (void)stream;
    return SKLTLT_ENOTSUP;
}
