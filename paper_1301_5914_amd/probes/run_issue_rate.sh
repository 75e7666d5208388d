#!/bin/bash
# Builds and runs the VALU issue-rate probe (issue_rate.hip) for gfx950; prints its table.
# Usage: bash paper_1301_5914_amd/probes/run_issue_rate.sh [output-dir]
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${1:-$here/_build}"
mkdir -p "$out"
/opt/rocm/bin/hipcc -O3 -std=c++17 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
    -Wno-unused-command-line-argument "$here/issue_rate.hip" -o "$out/issue_rate"
"$out/issue_rate"
/opt/rocm/bin/hipcc -O3 -std=c++17 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
    -Wno-unused-command-line-argument "$here/rsq_f64_accuracy.hip" -o "$out/rsq_f64_accuracy"
"$out/rsq_f64_accuracy"
