#include "sht.h"
#include "sht_internal.h"

extern "C" {
int sht_host_plan_create(int, int, const sht_plan_opts *, sht_host_plan_t **out) {
    if (out) *out = nullptr;
    return SHT_ERR_UNSUPPORTED;
}
void sht_host_plan_destroy(sht_host_plan_t *) {}
int sht_host_plan_apply(const sht_host_plan_t *, int, int, int, int, const double *, double *) {
    return SHT_ERR_UNSUPPORTED;
}
int sht_host_alt_matrix(const sht_host_plan_t *, int, int, double *) { return SHT_ERR_UNSUPPORTED; }
int sht_host_plan_stats(const sht_host_plan_t *, char *, size_t) { return SHT_ERR_UNSUPPORTED; }
}
