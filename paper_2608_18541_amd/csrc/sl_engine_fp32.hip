// sl_engine_fp32.hip -- the engine and its kernels instantiated for single-precision storage.
#include "sl_engine.hpp"

namespace slrt {

template class EngineT<float>;

Engine* make_engine_fp32(int max_runs) { return new EngineT<float>(max_runs); }

}  // namespace slrt
