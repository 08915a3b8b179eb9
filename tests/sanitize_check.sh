#!/bin/bash
# CPU sanitizer run: the FP64 oracle and the host side of the C boundary
# (argument validation, plan building, error paths) under AddressSanitizer
# and UndefinedBehaviorSanitizer, through the whole CPU test suite.
#   bash tests/sanitize_check.sh
# Needs the plain build first (python -c "import __graft_entry__ as g; g.build()").
set -e
cd "$(dirname "$0")/.."
python oracle/build.py --sanitize
python -m paper_2207_03530_amd.build --sanitize
ASAN_RT=$(gcc -print-file-name=libasan.so)
UBSAN_RT=$(gcc -print-file-name=libubsan.so)
LD_PRELOAD="$ASAN_RT $UBSAN_RT" \
ASAN_OPTIONS=detect_leaks=0:halt_on_error=1:abort_on_error=1 \
UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
VMAS_ORACLE_LIB=oracle/liboracle_san.so VMAS_LIB=paper_2207_03530_amd/libvmas_san.so \
python -m pytest tests -m "not gpu" -q -p no:xdist "$@"
