// Learned warm start (U-Net) -- model container; kernels follow.
#include <string>

#include "../../include/ni.h"
#include "ni_common.h"

namespace nil {

struct UnetModel {
  int dummy;
};

size_t unet_workspace_bytes(int H, int W) { return 256; }

int unet_load(UnetModel** out, const void* blob, size_t nbytes, std::string* err) {
  *out = nullptr;
  *err = "warm-start model format not supported by this build";
  return 0;
}

void unet_free(UnetModel* m) { delete m; }

hipError_t unet_predict(UnetModel* m, const float* normals, const uint8_t* mask, int H, int W, const ni_camera* cam,
                        float* out, void* ws, size_t wsb, hipStream_t st) {
  return hipErrorNotSupported;
}

}  // namespace nil
