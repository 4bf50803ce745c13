"""The profile summaries' kernel naming and source digest, on the CPU.

rocprofv3 records demangled kernel names; the summaries shorten them to the kernel's own
name, keep the batched path's instantiations (template argument Many) apart, and record a
digest of the kernel sources that changes with the code but not with its comments."""
from paper_2305_14306_amd import profile_report as pr

NS = "hav::(anonymous namespace)::"


def test_short_names():
    cases = {
        f"void {NS}k_bin_count<{NS}One>({NS}One)": "k_bin_count",
        f"void {NS}k_bin_count<{NS}Many>({NS}Many)": "k_bin_count (batch)",
        f"void {NS}k_bin_scatter<{NS}One, 512>({NS}One)": "k_bin_scatter",
        f"void {NS}k_bin_scatter<{NS}Many, 256>({NS}Many)": "k_bin_scatter (batch)",
        f"void {NS}k_select<{NS}Many>({NS}Many, int)": "k_select (batch)",
        f"{NS}k_search({NS}One, int, int)": "k_search",
        f"{NS}k_search_many({NS}Many, int)": "k_search_many",
        f"{NS}k_ws_init({NS}Ws, unsigned long)": "k_ws_init",
        "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)": "calib_neg (torch elementwise)",
        "void at::native::vectorized_elementwise_kernel<16, at::native::FillFunctor<unsigned char>>(int)": "torch fill",
    }
    for name, want in cases.items():
        assert pr.short_name(name) == want, (name, pr.short_name(name))


def test_digest_ignores_comments_only():
    code = "int a = 1;  // one\n// a whole comment line\nint b = 2;\n"
    same = "int a = 1;\nint b = 2;  // two\n"
    other = "int a = 1;\nint b = 3;\n"
    assert pr._code_only(code) == pr._code_only(same)
    assert pr._code_only(code) != pr._code_only(other)
    assert len(pr.source_digest()) == 16
