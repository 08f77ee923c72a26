// Batches of uneven pairs and the autotuner (placeholders until implemented).
#include "net.h"

extern "C" {

struct sv_batch_plan { int unused; };

sv_status sv_batch_plan_create(const sv_vae_desc *, int, int, int, int, int, int, sv_batch_plan **plan) {
    if (plan) *plan = nullptr;
    return SV_ERR_UNSUPPORTED;
}
sv_status sv_batch_plan_destroy(sv_batch_plan *) { return SV_OK; }
sv_status sv_stereo_batch(sv_batch_plan *, const sv_pair *, int, const void *, void *) { return SV_ERR_UNSUPPORTED; }
sv_status sv_autotune(const sv_vae_desc *, int, int, int, int, int, int) { return SV_ERR_UNSUPPORTED; }
sv_status sv_tile_config(int, char *buf, int buflen) {
    if (buf && buflen > 0) buf[0] = 0;
    return SV_ERR_UNSUPPORTED;
}

}
