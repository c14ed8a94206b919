// IIIB placeholder (filled in below).
#include "common.hpp"

namespace knnj {

knnj_status launch_iiib(Index* ix, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, int32_t* ids, void* sc,
                        int32_t* cnt, uint64_t* slots, hipStream_t st) {
  (void)ix; (void)R; (void)k; (void)opt; (void)ids; (void)sc; (void)cnt; (void)slots; (void)st;
  return fail(KNNJ_EUNSUPPORTED, "IIIB not built yet");
}

}  // namespace knnj
