// Autoencoder entry points (placeholder until the MFMA kernels land).
#include "ae_internal.h"

struct ae_net { int dummy; };

namespace wv {
int ae_latent_dim(const ae_net*) { throw Error{WV_ESTATE, "autoencoder not built"}; }
long long ae_latent_bytes_per_patch(const ae_net*, int) { throw Error{WV_ESTATE, "autoencoder not built"}; }
void ae_encode_state(const ae_net*, const PatchGrid&, const float*, int, void*, float*, float*, hipStream_t)
{ throw Error{WV_ESTATE, "autoencoder not built"}; }
void ae_decode_state(const ae_net*, const PatchGrid&, const void*, const float*, const float*, int, uint32_t,
                     float*, hipStream_t)
{ throw Error{WV_ESTATE, "autoencoder not built"}; }
}

extern "C" {
#define WV_STUB { wv::set_error("autoencoder not built"); return WV_ESTATE; }
int ae_create(int32_t, int32_t, int32_t, const float*, const double*, ae_net**) WV_STUB
void ae_destroy(ae_net*) {}
int ae_param_count(const ae_net*, int64_t*) WV_STUB
int ae_get_params(const ae_net*, float*) WV_STUB
int ae_set_params(ae_net*, const float*) WV_STUB
int ae_set_beta(ae_net*, const double*) WV_STUB
int ae_get_beta(const ae_net*, double*) WV_STUB
int ae_fit_beta(ae_net*, const wv_grid*, const float*, int64_t, double, void*) WV_STUB
int ae_save(const ae_net*, const char*) WV_STUB
int ae_load(const char*, ae_net**) WV_STUB
int ae_normalize(const ae_net*, const wv_grid*, const float*, uint16_t*, float*, void*) WV_STUB
int ae_encode(const ae_net*, const wv_grid*, const float*, int, void*, float*, float*, void*) WV_STUB
int ae_decode(const ae_net*, const wv_grid*, const void*, const float*, const float*, int, uint32_t, float*, void*) WV_STUB
int ae_train(ae_net*, const uint16_t*, int64_t, const ae_train_cfg*, const int32_t*, float*, void*) WV_STUB
int ae_train_step(ae_net*, const uint16_t*, const int32_t*, int32_t, double, const ae_train_cfg*, float*, double*, void*) WV_STUB
}
