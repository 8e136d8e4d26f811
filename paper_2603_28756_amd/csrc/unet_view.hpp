// What the reconstruction plan needs to know of a network (unet_api.cpp) to run the learned
// start: image size, batch limit, readiness, training domain and stream.
#pragma once

#include <hip/hip_runtime.h>

#include "tomo_nn.h"

namespace tomo {

struct UnetView {
  int height = 0, width = 0, max_batch = 0;
  bool ready = false;       // workspace attached and parameters set
  bool has_domain = false;
  tomo_unet_domain_t domain{};
  hipStream_t stream = nullptr;
};

bool unet_view(tomo_unet net, UnetView* out);

}  // namespace tomo
