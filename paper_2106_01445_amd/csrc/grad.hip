#include "internal.h"
int approx_backward(gbs_ctx *ctx, gbs_plan *, const double *, double *, double *)
{
    return set_err(ctx, -1, "gradient not built yet");
}
