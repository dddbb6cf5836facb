// MFMA derivation (BF16 / FP8-weight forms).
#include "gsc_derive_mfma.h"

namespace gsc {

hipError_t derive_mfma(const MfmaDeriveArgs&, int64_t, hipStream_t) { return hipErrorNotSupported; }

}  // namespace gsc
