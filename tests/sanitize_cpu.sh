#!/bin/bash
# The CPU test suite with the host code under AddressSanitizer and
# UndefinedBehaviorSanitizer: the oracle's C (clang) and the library's host
# C++ (hipcc, sanitizers on the host pass only; device code is unchanged),
# both built into a temporary directory and loaded through MRIP_ORACLE_LIB /
# MRIP_LIB, with the clang ASan runtime preloaded into Python.
#   bash tests/sanitize_cpu.sh [extra pytest args]
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
OUT="$(mktemp -d /tmp/mrip_san.XXXXXX)"
LLVM=/opt/rocm/llvm
RT="$(ls $LLVM/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)"
SAN="-fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer -g"
$LLVM/bin/clang -O1 $SAN -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math \
  "$ROOT/oracle/oracle.c" -o "$OUT/liboracle.so" -lm
HOST=""
for f in $SAN; do HOST="$HOST -Xarch_host $f"; done
/opt/rocm/bin/hipcc -O1 -std=c++17 --offload-arch=gfx950 -fPIC -shared -ffp-contract=off \
  -fno-fast-math -fvisibility=hidden -Xclang -target-feature -Xclang -packed-fp32-ops \
  -I"$ROOT/include" $HOST "$ROOT"/paper_1501_01405_amd/csrc/*.hip \
  "$ROOT"/paper_1501_01405_amd/csrc/*.cpp -o "$OUT/libmrip.so" 2>&1 | grep -v packed-fp32 || true
test -f "$OUT/libmrip.so"
cd "$ROOT"
MRIP_LIB="$OUT/libmrip.so" MRIP_ORACLE_LIB="$OUT/liboracle.so" LD_PRELOAD="$RT" \
  ASAN_OPTIONS=detect_leaks=0:detect_odr_violation=0:verify_asan_link_order=0:halt_on_error=1:log_path=${SAN_LOG:-/tmp/mrip_san} \
  UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1:log_path=${SAN_LOG:-/tmp/mrip_san} \
  python -m pytest tests -m "not gpu" -q -p no:xdist -p no:cacheprovider "$@"
