// rs_batched.hip -- many independent arrays in one launch sequence.
#include "rs_internal.h"

using namespace rs;

extern "C" {

rs_status rs_batched_temp_bytes(const rs_key_desc *desc, uint64_t total, uint32_t nseg, int with_values,
                                size_t *bytes) {
  (void)desc; (void)total; (void)nseg; (void)with_values; (void)bytes;
  return fail(RS_ERR_UNSUPPORTED, "batched sort not built yet");
}

rs_status rs_sort_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                          uint32_t *vals_out, const uint64_t *d_seg_offsets, uint32_t nseg, uint64_t total, void *tmp,
                          size_t tmp_bytes, void *stream) {
  (void)desc; (void)keys_in; (void)keys_out; (void)vals_in; (void)vals_out; (void)d_seg_offsets; (void)nseg;
  (void)total; (void)tmp; (void)tmp_bytes; (void)stream;
  return fail(RS_ERR_UNSUPPORTED, "batched sort not built yet");
}

}
