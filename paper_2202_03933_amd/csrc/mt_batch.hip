// Batched evaluation of many interfaces: placeholder entry points.
#include "mt_internal.h"

extern "C" {
int mt_batch_create(mt_batch** b, int device) { (void)b; (void)device; mt::set_error("batch: not built"); return MT_EUNSUPPORTED; }
int mt_batch_destroy(mt_batch* b) { (void)b; return MT_OK; }
int mt_batch_add(mt_batch* b, mt_ctx* c, int32_t* i) { (void)b; (void)c; (void)i; return MT_EUNSUPPORTED; }
int mt_batch_build(mt_batch* b, const mt_batch_tuning* t, void* s) { (void)b; (void)t; (void)s; return MT_EUNSUPPORTED; }
int mt_batch_forward(mt_batch* b, double* const* D, double* const* M, double* const* g, int ug, void* s) {
  (void)b; (void)D; (void)M; (void)g; (void)ug; (void)s; return MT_EUNSUPPORTED; }
int mt_batch_backward(mt_batch* b, const double* const* WD, const double* const* WM, const double* const* wg,
                      double* const* gs, double* const* gm, int ug, void* s) {
  (void)b; (void)WD; (void)WM; (void)wg; (void)gs; (void)gm; (void)ug; (void)s; return MT_EUNSUPPORTED; }
int mt_batch_autotune(mt_batch* b, mt_batch_tuning* o, void* s) { (void)b; (void)o; (void)s; return MT_EUNSUPPORTED; }
}
