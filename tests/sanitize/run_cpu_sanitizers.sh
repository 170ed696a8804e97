#!/bin/bash
# CPU-only AddressSanitizer + UndefinedBehaviorSanitizer run of the oracle and of the library's
# host runtime (no GPU needed; the device code is built as usual).
#   1. the 2-D and 3-D oracles built with g++ -fsanitize=address,undefined, then the oracle
#      pins (tests/test_oracle_pins.py, tests/test_oracle3d_pins.py) against them;
#   2. the library built with the host side instrumented (clang, -Xarch_host), then the CPU
#      tests of the C ABI (tests/test_abi.py: validation, host fits, the film inversion).
# Builds go to a temporary directory; the in-tree libraries are not touched.
# Usage: bash tests/sanitize/run_cpu_sanitizers.sh
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/../.." && pwd)"
OUT="$(mktemp -d)"
SAN="-fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer -g"
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1

echo "== oracle (g++ $SAN)"
for src in lb_oracle lb_oracle3d; do
  g++ -O1 -std=c++17 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math $SAN \
      "$ROOT/oracle/$src.cpp" -o "$OUT/lib$src.so"
done
LD_PRELOAD="$(g++ -print-file-name=libasan.so):$(g++ -print-file-name=libubsan.so)" \
LB_ORACLE_LIB_DIR="$OUT" OMP_NUM_THREADS=2 \
  python3 -m pytest -x -q -m "not gpu and not slow" -p no:cacheprovider \
  "$ROOT/tests/test_oracle_pins.py" "$ROOT/tests/test_oracle3d_pins.py"

echo "== host runtime (hipcc, -Xarch_host sanitizers)"
CL_RT="$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)"
FL="--offload-arch=gfx950 -O1 -std=c++17 -fPIC -Xclang -target-feature -Xclang -packed-fp32-ops -ffp-contract=off -I$ROOT/include"
SRCS="lb_step_f64.hip lb_step_f32.hip lb_step_bf16.hip lb_kernels.hip lb_adjoint.hip lb_static.hip lb3_kernels.hip lb_api.cpp lb_batch.cpp lb_rheology.cpp lb3_api.cpp"
for f in $SRCS; do
  /opt/rocm/bin/hipcc $FL -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
      -Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer \
      -c "$ROOT/paper_1402_6019_amd/csrc/$f" -o "$OUT/${f%.*}.o" 2>/dev/null &
done
wait
# link step only: -fno-gpu-sanitize keeps the device code objects uninstrumented
/opt/rocm/bin/hipcc --offload-arch=gfx950 -shared -fPIC -fno-gpu-sanitize -fsanitize=address -fsanitize=undefined -shared-libsan \
    "$OUT"/*.o -o "$OUT/liblb355.so"
LD_PRELOAD="$CL_RT" LB355_LIB="$OUT/liblb355.so" \
  python3 -m pytest -x -q -m "not gpu" -p no:cacheprovider "$ROOT/tests/test_abi.py"
echo "sanitizer runs passed"
