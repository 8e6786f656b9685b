// sl_engine_fp64.hip -- the engine and its kernels instantiated for double-precision storage.
#include "sl_engine.hpp"

namespace slrt {

template class EngineT<double>;

Engine* make_engine_fp64(int max_runs) { return new EngineT<double>(max_runs); }

}  // namespace slrt
