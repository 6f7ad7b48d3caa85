#!/bin/bash
# Builds the host-audit program: the library's engine (host side instrumented
# by a sanitizer, pool audit hooks on), the kernels object of the regular
# build (its launch wrappers), the mock runtime and the driver.
#   build.sh OUTDIR address|thread
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
ROOT=$(cd "$HERE/../.." && pwd)
OUT=$1
SAN=${2:-address}
mkdir -p "$OUT"
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
CXX=${CXX_AUDIT:-/opt/rocm/llvm/bin/clang++}
SANF="-Xarch_host -fsanitize=$SAN -Xarch_host -fno-omit-frame-pointer"
KOBJ=$ROOT/paper_1309_5050_amd/_build/kernels.o
test -f "$KOBJ" || { echo "build the library first (its kernels object is linked)"; exit 3; }
"$HIPCC" --offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -DSHSSA_HOST_AUDIT $SANF \
    -Xclang -target-feature -Xclang -packed-fp32-ops \
    -c "$ROOT/paper_1309_5050_amd/csrc/engine.hip" -o "$OUT/engine_audit.o" 2> "$OUT/engine_build.log"
"$HIPCC" -x hip --cuda-host-only -O1 -g -std=c++17 -fPIC $SANF \
    -c "$HERE/mock_hip.cpp" -o "$OUT/mock_hip.o" 2> "$OUT/mock_build.log"
"$CXX" -O1 -g -std=c++17 -fsanitize=$SAN -fno-omit-frame-pointer -c "$HERE/driver.cpp" -o "$OUT/driver.o"
"$CXX" -fsanitize=$SAN "$OUT/engine_audit.o" "$KOBJ" "$OUT/mock_hip.o" "$OUT/driver.o" -o "$OUT/audit" -lpthread
echo "built $OUT/audit"
